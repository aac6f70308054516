// libexpm_pfd, banded route: R_d(tA)V for Hermitian band matrices (see
// include/expm_pfd.h, expm_pfd_band_*).
//
// The paper's experiments apply the method to finite-difference Laplacians
// (Sec. 5), for which every shifted matrix tA + theta_k I of eq. equ:expAx is a
// band matrix: each pole is one banded solve, O(n kd (kd + m)) work instead of a
// dense LU.  Gaussian elimination with partial pivoting inside the band: at
// column j the candidates are the kd + 1 rows not yet used as pivots whose band
// reaches column j, the pivot row (with up to 2 kd entries right of the diagonal
// after fill) becomes row j of U, and the elimination is applied to V at once;
// a banded back substitution follows.  Solutions of all poles are then summed
// with their residues in FP64 in a fixed order.
//
// Kernels:
//  k_band_narrow<KD> (kd <= 3): one wave per pole.  The elimination window (the
//    kd + 1 active rows over columns j .. j + 2kd) is the same in every lane and
//    lives in registers; each lane carries one right-hand side.  Row j of U, with
//    the reciprocal of its pivot in place of the diagonal, goes to memory; the
//    back substitution runs in the same wave, one lane per column, the last 2kd
//    solution values in registers.
//  k_band_factor<CPW> (kd >= 4): one workgroup per (pole, block of up to 16
//    right-hand sides).  Lane i of every wave holds active-row slot i; the window
//    columns (circular: column c in slot c mod (2kd + 1)) and the right-hand
//    sides are spread over the waves, CPW slots each.  Per column: the wave
//    holding the column finds the pivot (wave argmax) and the multipliers and
//    publishes them in LDS (two buffers, so one barrier per column suffices);
//    every wave then updates its slots against the pivot row (read with
//    readlane), the pivot row leaves as row j of U, and its lane takes the next
//    matrix row, loaded one column ahead.
//  k_band_back: banded back substitution, one wave per right-hand side; the last
//    128 solution values in a register ring (two per lane), each step's products
//    reduced across the wave.
//  k_band_accum: X = sum_k w_k Y_k in FP64, fixed pole order (w_k: residues
//    times e^c), or 2 Re(...) over one pole per pair for real data.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "host_common.h"
#include "band_chain.h"
#include "spike.h"

using namespace expm;

namespace {

constexpr int BAND_MC = 16;        // right-hand sides per workgroup of the wide-band kernels
constexpr int BAND_NARROW_KD = 3;  // widest band of the one-wave kernel (its window stays in registers)

struct BandDesc {
  const double2* AB;
  int64_t ldab;
  const double2* V;
  int64_t ldv;
  double t, c;  // c: shift in units of tA (subtracted from the diagonal)
  int n, kd, kw, m;  // kd: stored band; kw = min(kd, n - 1): the band worked on
  int real, upper;
};

// entry (i, col) of tA - cI; zero outside the matrix or the band
__device__ __forceinline__ double2 band_at(const BandDesc& b, int i, int col) {
  double2 v = czero<double2>();
  if (i < 0 || col < 0 || i >= b.n || col >= b.n) return v;
  const int off = i - col;
  if (off > b.kw || -off > b.kw) return v;
  if (b.upper)  // A(i, col) for i <= col at AB[kd + i - col, col]
    v = off <= 0 ? b.AB[(b.kd + off) + (int64_t)col * b.ldab] : cconj(b.AB[(b.kd - off) + (int64_t)i * b.ldab]);
  else  // A(i, col) for i >= col at AB[i - col, col]
    v = off >= 0 ? b.AB[off + (int64_t)col * b.ldab] : cconj(b.AB[-off + (int64_t)i * b.ldab]);
  if (off == 0) {
    v.x = b.t * v.x - b.c;
    v.y = 0.0;
    return v;
  }
  if (b.real) v.y = 0.0;
  v.x *= b.t;
  v.y *= b.t;
  return v;
}
// entry (i, col) of tA - cI + theta I
__device__ __forceinline__ double2 shifted_at(const BandDesc& b, double2 th, int i, int col) {
  double2 v = band_at(b, i, col);
  if (i == col && i < b.n) {
    v.x += th.x;
    v.y += th.y;
  }
  return v;
}
__device__ __forceinline__ double2 rhs_at(const BandDesc& b, int i, int r) {
  double2 v = czero<double2>();
  if (i < b.n && r < b.m) {
    v = b.V[i + (int64_t)r * b.ldv];
    if (b.real) v.y = 0.0;
  }
  return v;
}
// maximum over the wave of a 64-bit integer, returned in every lane
__device__ __forceinline__ long long wave_max_i64(long long x) {
  auto step = [](long long v, long long o) { return o > v ? o : v; };
  x = step(x, __double_as_longlong(dpp_move<0xB1, 0xF>(__longlong_as_double(x))));
  x = step(x, __double_as_longlong(dpp_move<0x4E, 0xF>(__longlong_as_double(x))));
  x = step(x, __double_as_longlong(dpp_move<0x141, 0xF>(__longlong_as_double(x))));
  x = step(x, __double_as_longlong(dpp_move<0x140, 0xF>(__longlong_as_double(x))));
  x = step(x, __double_as_longlong(dpp_move<0x142, 0xA>(__longlong_as_double(x))));
  x = step(x, __double_as_longlong(dpp_move<0x143, 0xC>(__longlong_as_double(x))));
  const int lo = __builtin_amdgcn_readlane((int)(x & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), 63);
  return ((long long)hi << 32) | (unsigned int)lo;
}

// sum over the wave, valid in lane 63 and returned in every lane
__device__ __forceinline__ double wave_sum_dpp(double x) {
  x += dpp_move<0xB1, 0xF>(x);
  x += dpp_move<0x4E, 0xF>(x);
  x += dpp_move<0x141, 0xF>(x);
  x += dpp_move<0x140, 0xF>(x);
  x += dpp_move<0x142, 0xA>(x);
  x += dpp_move<0x143, 0xC>(x);
  return lane_bcast(x, 63);
}

// Rows of tA - cI inside the band, row-major: R[q*W + c] = entry (q, q - kw + c)
// (zero outside the matrix), W = 2 kw + 1; and V row-major: Vr[q*m + r].  The
// chains below read both front to back in whole 64-value chunks.
__global__ __launch_bounds__(256) void k_band_rows(BandDesc b, double2* __restrict__ R, double2* __restrict__ Vr) {
  const int W = 2 * b.kw + 1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)b.n * W; e += stride) {
    const int q = (int)(e / W), c = (int)(e % W);
    R[e] = band_at(b, q, q - b.kw + c);
  }
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)b.n * b.m; e += stride)
    Vr[e] = rhs_at(b, (int)(e / b.m), (int)(e % b.m));
}

// ---- wide bands: one workgroup per (pole, block of right-hand sides) ----------
// Same U and Y layouts as the narrow kernel (W = 2 kw + 1; one U copy, written by
// the first block of right-hand sides).  Block-staged like the narrow kernel: the
// rows inserted during a block of WB_B columns (R and V) sit in LDS, and the rows
// of U and Y it produces collect in LDS until the block boundary.
constexpr int WB_B = 16;                                   // columns per block
constexpr int WB_ROW = 2 * EXPM_PFD_BAND_MAX_KD + 1 + BAND_MC;  // largest staged row
constexpr int WB_G = 5;  // staging values per thread (16 rows x 143 over >= 448 threads)
template <int CPW>
__global__ __launch_bounds__(512) void k_band_factor(int n, int kw, int m, const double2* __restrict__ R,
                                                     const double2* __restrict__ Vr,
                                                     const double2* __restrict__ pole, double2* __restrict__ U,
                                                     double2* __restrict__ Y, int64_t ustride, int64_t ystride) {
  __shared__ double2 lbuf[2][64];
  __shared__ int pbuf[2];
  __shared__ double2 sIn[WB_B * WB_ROW], sOut[WB_B * WB_ROW], sRinv[2][WB_B];
  const int k = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int NW = blockDim.x >> 6, NT = blockDim.x;
  const int W = 2 * kw + 1;
  const int r0 = blockIdx.y * BAND_MC, mc = min(BAND_MC, m - r0);
  const int slots = W + mc, RW = W + BAND_MC;  // RW: staged row length
  const bool writeU = blockIdx.y == 0;
  const double2 th = pole[k];
  double2* Uk = U + k * ustride;
  double2* Yk = Y + k * ystride;
  const int nblk = (n + WB_B - 1) / WB_B;

  double2 g[WB_G];
  // staged row i of block b: matrix row q = b*B + kw + 1 + i: R entries, then V
  auto load_in = [&](int b) {
#pragma unroll
    for (int c = 0; c < WB_G; ++c) {
      const int f = tid + c * NT, i = f / RW, e = f % RW;
      const int64_t q = (int64_t)b * WB_B + kw + 1 + i;
      g[c] = czero<double2>();
      if (f < WB_B * RW && q < n) {
        if (e < W) g[c] = R[q * W + e];
        else if (e - W < mc) g[c] = Vr[q * m + r0 + e - W];
      }
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int c = 0; c < WB_G; ++c) {
      const int f = tid + c * NT;
      if (f < WB_B * RW) sIn[f] = g[c];
    }
  };
  auto flush = [&](int b) {  // rows of block b from sOut and sRinv
    const int j0 = b * WB_B, rows = min(WB_B, n - j0);
#pragma unroll
    for (int c = 0; c < WB_G; ++c) {
      const int f = tid + c * NT, i = f / RW, e = f % RW;
      if (f < WB_B * RW && i < rows) {
        const int64_t j = j0 + i;
        if (e < W) {
          if (writeU) Uk[j * W + e] = e == 0 ? sRinv[b & 1][i] : sOut[f];
        } else if (e - W < mc) {
          Yk[j * m + r0 + e - W] = sOut[f];
        }
      }
    }
  };

  double2 a[CPW];
  bool alive = lane <= kw && lane < n;  // active-row slot `lane` holds matrix row `lane`
  // window at column 0: slot s holds column s; right-hand side slots W + r
#pragma unroll
  for (int i = 0; i < CPW; ++i) {
    const int s = wv + i * NW;
    a[i] = czero<double2>();
    if (alive && s < W) {
      const int off = s - lane + kw;
      if (off >= 0 && off < W) {
        a[i] = R[(int64_t)lane * W + off];
        if (off == kw) {
          a[i].x += th.x;
          a[i].y += th.y;
        }
      }
    } else if (alive && s < slots) {
      a[i] = Vr[(int64_t)lane * m + r0 + s - W];
    }
  }
  // pivot and multipliers of column j, held in z (run by the wave holding it)
  auto pivot = [&](double2 z, int nb, int j) {
    // one reduction over keys: the magnitude's bits (a non-negative double orders
    // as an integer) with the low 6 bits replaced by 63 - lane, so the largest key
    // is a largest magnitude (to 2^-46 relative) at the lowest such lane
    long long key = -1;
    if (alive) key = (__double_as_longlong(pivot_mag(z)) & ~63ll) | (63 - lane);
    const int pl = 63 - (int)(wave_max_i64(key) & 63);
    const double2 piv = lane_bcast2(z, pl);
    const double2 rp = crecip_fast(piv);
    lbuf[nb][lane] = (alive && lane != pl) ? cmul(z, rp) : czero<double2>();
    if (lane == 0) {
      pbuf[nb] = pl;
      sRinv[(j / WB_B) & 1][j % WB_B] = rp;
    }
  };
#pragma unroll
  for (int i = 0; i < CPW; ++i)
    if (wv + i * NW == 0) pivot(a[i], 0, 0);
  load_in(0);
  for (int b = 0; b < nblk; ++b) {
    lds_barrier();  // the last block's reads of sIn and writes of sOut are done
    stage();
    if (b > 0) flush(b - 1);
    if (b + 1 < nblk) load_in(b + 1);
    lds_barrier();
    const int j0 = b * WB_B, jn = min(WB_B, n - j0);
    for (int jj = 0; jj < jn; ++jj) {
      const int j = j0 + jj;
      const int buf = j & 1;
      const int p = __builtin_amdgcn_readfirstlane(pbuf[buf]);
      const double2 l = lbuf[buf][lane];
      const bool qin = j + kw + 1 < n;
      const int sj = j % W;        // slot of column j: it leaves, and takes column j + W
      const int s1 = (j + 1) % W;  // slot of column j + 1
      const double2* in = sIn + jj * RW;
      double2* out = sOut + jj * RW;
#pragma unroll
      for (int i = 0; i < CPW; ++i) {
        const int s = wv + i * NW;
        if (s >= slots) continue;
        const double2 pv = lane_bcast2(a[i], p);
        if (s < W) {
          const int cofs = s >= sj ? s - sj : s - sj + W;  // column - j
          if (lane == p) {
            if (cofs > 0) out[cofs] = a[i];
            // the new row's entry at this slot's column in step j + 1
            const int e1 = s >= s1 ? s - s1 : s - s1 + W;
            a[i] = qin ? in[e1] : czero<double2>();
            if (qin && e1 == kw) {
              a[i].x += th.x;
              a[i].y += th.y;
            }
          } else {
            // column j + W is zero in the remaining rows (they end before it)
            a[i] = cofs == 0 ? czero<double2>() : cfms(a[i], l, pv);
          }
        } else {
          if (lane == p) {
            out[s] = a[i];
            a[i] = qin ? in[s] : czero<double2>();
          } else {
            a[i] = cfms(a[i], l, pv);
          }
        }
      }
      if (lane == p) alive = qin;
      if (j + 1 < n) {
#pragma unroll
        for (int i = 0; i < CPW; ++i)
          if (wv + i * NW == s1) pivot(a[i], buf ^ 1, j + 1);
      }
      lds_barrier();
    }
  }
  flush(nblk - 1);
}

// back substitution x_j = (1/u_jj) (y_j - sum_{c=1..2kw} u_{j,j+c} x_{j+c}), in place
// in Y; one wave per right-hand side (at least four waves, for the staging).  The
// ring holds x_i at position i mod 128 (positions lane and lane + 64); blocks of
// WB_B rows of U and y are staged in LDS a block ahead, and the block's x rows are
// written back at the next boundary.
constexpr int BK_G = 8;  // staging values per thread (16 rows x 127 over >= 256 threads)
__global__ __launch_bounds__(1024) void k_band_back(int n, int kw, int m, const double2* __restrict__ U,
                                                    double2* __restrict__ Y, int64_t ustride, int64_t ystride) {
  __shared__ double2 sU[WB_B * (2 * EXPM_PFD_BAND_MAX_KD + 1)], sYin[BAND_MC][WB_B], sX[BAND_MC][WB_B];
  const int k = blockIdx.x, tid = threadIdx.x, lane = tid & 63, NT = blockDim.x;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r0 = blockIdx.y * BAND_MC, mc = min(BAND_MC, m - r0);
  const bool act = wv < mc;
  const int W = 2 * kw + 1;
  const double2* Uk = U + k * ustride;
  double2* Yk = Y + k * ystride;
  const int nblk = (n + WB_B - 1) / WB_B;
  double2 g[BK_G], gy;
  auto load_in = [&](int b) {
    const int j0 = b * WB_B, rows = min(WB_B, n - j0);
#pragma unroll
    for (int c = 0; c < BK_G; ++c) {
      const int f = tid + c * NT;
      g[c] = f < rows * W ? Uk[(int64_t)j0 * W + f] : czero<double2>();
    }
    const int i = tid / BAND_MC, cc = tid % BAND_MC;
    gy = (i < rows && cc < mc) ? Yk[(int64_t)(j0 + i) * m + r0 + cc] : czero<double2>();
  };
  auto stage = [&]() {
#pragma unroll
    for (int c = 0; c < BK_G; ++c) {
      const int f = tid + c * NT;
      if (f < WB_B * W) sU[f] = g[c];
    }
    const int i = tid / BAND_MC, cc = tid % BAND_MC;
    if (i < WB_B) sYin[cc][i] = gy;
  };
  auto flush = [&](int b) {
    const int j0 = b * WB_B, rows = min(WB_B, n - j0);
    const int i = tid / BAND_MC, cc = tid % BAND_MC;
    if (i < rows && cc < mc) Yk[(int64_t)(j0 + i) * m + r0 + cc] = sX[cc][i];
  };
  double2 x0 = czero<double2>(), x1 = czero<double2>();
  load_in(nblk - 1);
  for (int b = nblk - 1; b >= 0; --b) {
    lds_barrier();
    stage();
    if (b + 1 < nblk) flush(b + 1);
    if (b > 0) load_in(b - 1);
    lds_barrier();
    const int j0 = b * WB_B, jn = min(WB_B, n - j0);
    if (act) {
      for (int jj = jn - 1; jj >= 0; --jj) {
        const int j = j0 + jj;
        const int c0 = (lane - j) & 127, c1 = (lane + 64 - j) & 127;
        const double2 u0 = (c0 >= 1 && c0 < W && j + c0 < n) ? sU[jj * W + c0] : czero<double2>();
        const double2 u1 = (c1 >= 1 && c1 < W && j + c1 < n) ? sU[jj * W + c1] : czero<double2>();
        double2 t = cmul(u0, x0);
        t.x += u1.x * x1.x - u1.y * x1.y;
        t.y += u1.x * x1.y + u1.y * x1.x;
        const double2 y = sYin[wv][jj];
        double2 s;
        s.x = y.x - wave_sum_dpp(t.x);
        s.y = y.y - wave_sum_dpp(t.y);
        const double2 x = cmul(sU[jj * W], s);
        if ((j & 63) == lane) {
          if (j & 64) x1 = x;
          else x0 = x;
        }
        if (lane == 0) sX[wv][jj] = x;
      }
    }
  }
  lds_barrier();
  flush(0);
}

// X(:, r) = sum_k w_k Y_k(:, r) over the S solves in order (real: 2 Re(...))
__global__ __launch_bounds__(256) void k_band_accum(int n, int m, int S, int real, const double2* __restrict__ w,
                                                    double ec, const double2* __restrict__ Y, int64_t ystride,
                                                    double2* __restrict__ X, int64_t ldx) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)n * m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / n), j = (int)(e % n);
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < S; ++k) {
      double2 a = w[k];
      a.x *= ec;
      a.y *= ec;
      const double2 y = Y[k * ystride + (int64_t)j * m + r];
      sr += a.x * y.x - a.y * y.y;
      si += a.x * y.y + a.y * y.x;
    }
    X[j + (int64_t)r * ldx] = real ? double2{2.0 * sr, 0.0} : double2{sr, si};
  }
}

int grid_for(int64_t count) {
  const int64_t g = (count + 255) / 256;
  return (int)std::min<int64_t>(std::max<int64_t>(g, 1), 65536);
}

}  // namespace

struct expm_pfd_band_s {
  int64_t n = 0, kd = 0, kw = 0, m_max = 0;
  int degree = 0, S = 0;  // S: solves per apply (d, or d/2 with real data)
  int real = 0, upper = 0, shift_t = 0;
  double shift = 0.0;
  int64_t ustride = 0, ystride = 0;
  double2* pole = nullptr;  // S poles theta_k (pair representatives, then their conjugates)
  double2* w = nullptr;     // S residues
  double2* U = nullptr;
  double2* Y = nullptr;
  double2* R = nullptr;   // n x (2 kw + 1): rows of tA - cI inside the band
  double2* Vr = nullptr;  // n x m_max: V row-major
  double2* spk = nullptr;  // kd = 1 from order SPIKE_MIN_N: the spike solver's workspace (no U)
};

namespace {
void band_free(expm_pfd_band_t p) {
  if (!p) return;
  void* ptrs[] = {p->pole, p->w, p->U, p->Y, p->R, p->Vr, p->spk};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete p;
}
}  // namespace

extern "C" int expm_pfd_band_plan(expm_pfd_band_t* out, int64_t n, int64_t kd, int degree, int64_t m_max,
                                  const expm_pfd_opts* opts) {
  if (!out) return EXPM_PFD_ERR_NULL;
  *out = nullptr;
  if (int e = check_degree(degree)) return e;
  if (n < 1 || n > EXPM_PFD_BAND_MAX_N || kd < 0 || kd > EXPM_PFD_BAND_MAX_KD || m_max < 1 || m_max > 64)
    return EXPM_PFD_ERR_DIM;
  if (int e = check_opts(opts)) return e;
  const int P = degree / 2;
  std::vector<double2> th(P), a(P);
  if (int rc = expm_pfd_constants(degree, (double*)th.data(), (double*)a.data())) return rc;
  auto* p = new expm_pfd_band_s();
  p->n = n;
  p->kd = kd;
  p->kw = std::min<int64_t>(kd, n - 1);
  p->m_max = m_max;
  p->degree = degree;
  p->real = opts && opts->real_data ? 1 : 0;
  p->upper = opts ? opts->uplo : 0;
  p->shift = opts ? opts->shift : 0.0;
  p->shift_t = opts && opts->shift_scale_t ? 1 : 0;
  p->S = p->real ? P : 2 * P;
  std::vector<double2> hp(p->S), hw(p->S);
  for (int k = 0; k < P; ++k) {
    hp[k] = th[k];
    hw[k] = a[k];
    if (!p->real) {
      hp[P + k] = double2{th[k].x, -th[k].y};
      hw[P + k] = double2{a[k].x, -a[k].y};
    }
  }
  const int64_t W = 2 * p->kw + 1;
  // the one-wave kernel keeps a copy of U per block of 16 right-hand sides
  const int64_t ucopies = p->kw <= BAND_NARROW_KD ? (m_max + NB_MC - 1) / NB_MC : 1;
  p->ustride = n * W;
  p->ystride = n * m_max;
  const bool spike = p->kw == 1 && n >= SPIKE_MIN_N;
  bool ok = hipMalloc((void**)&p->pole, p->S * sizeof(double2)) == hipSuccess &&
            hipMalloc((void**)&p->w, p->S * sizeof(double2)) == hipSuccess &&
            (spike || hipMalloc((void**)&p->U, (size_t)p->S * ucopies * p->ustride * sizeof(double2)) == hipSuccess) &&
            hipMalloc((void**)&p->Y, (size_t)p->S * p->ystride * sizeof(double2)) == hipSuccess &&
            hipMalloc((void**)&p->R, (size_t)n * W * sizeof(double2)) == hipSuccess &&
            hipMalloc((void**)&p->Vr, (size_t)n * m_max * sizeof(double2)) == hipSuccess;
  if (ok && spike) {
    const SpikePlan q = spike_plan(n, p->S, (int)m_max);
    ok = hipMalloc((void**)&p->spk, spike_bytes(q, p->S)) == hipSuccess &&
         hipMemset(p->spk, 0, (size_t)p->S * sizeof(double2)) == hipSuccess;  // the zero poles
  }
  ok = ok && hipMemcpy(p->pole, hp.data(), p->S * sizeof(double2), hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(p->w, hw.data(), p->S * sizeof(double2), hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    const bool oom = hipGetLastError() == hipErrorOutOfMemory;
    band_free(p);
    return oom ? EXPM_PFD_ERR_OOM : EXPM_PFD_ERR_HIP;
  }
  *out = p;
  return 0;
}

namespace {
template <int CPW>
void launch_factor(dim3 grid, int nw, hipStream_t st, const BandDesc& bd, expm_pfd_band_t p) {
  hipLaunchKernelGGL(k_band_factor<CPW>, grid, dim3(64 * nw), 0, st, bd.n, bd.kw, bd.m, p->R, p->Vr, p->pole, p->U,
                     p->Y, p->ustride, p->ystride);
}
}  // namespace

extern "C" int expm_pfd_band_apply(expm_pfd_band_t p, double t, const void* AB, int64_t ldab, const void* V,
                                   int64_t ldv, int64_t m, void* X, int64_t ldx, void* stream) {
  if (!p || !AB || !V || !X) return EXPM_PFD_ERR_NULL;
  if (!std::isfinite(t)) return EXPM_PFD_ERR_ARG;
  if (m < 1 || m > p->m_max) return EXPM_PFD_ERR_DIM;
  if (ldab < p->kd + 1 || ldv < p->n || ldx < p->n) return EXPM_PFD_ERR_LD;
  ProblemDesc sh{};
  if (problem_shift(p->shift, p->shift_t, t, sh)) return EXPM_PFD_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  BandDesc bd;
  bd.AB = (const double2*)AB;
  bd.ldab = ldab;
  bd.V = (const double2*)V;
  bd.ldv = ldv;
  bd.t = t;
  bd.c = sh.c;
  bd.n = (int)p->n;
  bd.kd = (int)p->kd;
  bd.kw = (int)p->kw;
  bd.m = (int)m;
  bd.real = p->real;
  bd.upper = p->upper;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_band_rows, dim3(grid_for(p->n * (2 * p->kw + 1))), dim3(256), 0, st, bd, p->R, p->Vr);
  const dim3 g1((unsigned)p->S, (unsigned)((m + NB_MC - 1) / NB_MC));
  const int n = bd.n, mm = bd.m;
  if (p->spk) {
    SpikeSrc src{};
    src.kind = 0;
    src.R = p->R;
    src.V = p->Vr;
    src.mv = mm;
    src.ncol = mm;
    src.n = n;
    const SpikePlan q = spike_plan(n, p->S, mm);
    spike_solve(src, p->pole, p->S, q, spike_carve(p->spk, q, p->S), SpikeOutRows{p->Y, p->ystride, mm}, st);
  } else if (p->kw <= BAND_NARROW_KD) {
#define EXPM_BAND_NARROW(KD) \
  hipLaunchKernelGGL(k_band_narrow<KD>, g1, dim3(64), 0, st, n, mm, p->R, p->Vr, p->pole, p->U, p->Y, p->ustride, \
                     p->ystride, (int64_t)0, (int64_t)0)
    switch (p->kw) {
      case 0: EXPM_BAND_NARROW(0); break;
      case 1: EXPM_BAND_NARROW(1); break;
      case 2: EXPM_BAND_NARROW(2); break;
      default: EXPM_BAND_NARROW(3); break;
    }
#undef EXPM_BAND_NARROW
  } else {
    const int chunks = (int)((m + BAND_MC - 1) / BAND_MC);
    const int slots = (int)(2 * p->kw + 1 + std::min<int64_t>(BAND_MC, m));
    // fewest slots per wave that keep the workgroup within 8 waves
    const int cpw = slots <= 16 ? 2 : slots <= 32 ? 4 : slots <= 64 ? 8 : slots <= 96 ? 12 : 18;
    // enough waves for the slots, and for staging a block of rows (WB_G values per thread)
    const int stage_w = (int)((WB_B * (2 * p->kw + 1 + BAND_MC) + 64 * WB_G - 1) / (64 * WB_G));
    const int nw = std::max((slots + cpw - 1) / cpw, stage_w);
    if (nw > 8) return EXPM_PFD_ERR_HIP;  // (cannot happen: kw <= 63)
    const dim3 grid((unsigned)p->S, (unsigned)chunks);
    switch (cpw) {
      case 2: launch_factor<2>(grid, nw, st, bd, p); break;
      case 4: launch_factor<4>(grid, nw, st, bd, p); break;
      case 8: launch_factor<8>(grid, nw, st, bd, p); break;
      case 12: launch_factor<12>(grid, nw, st, bd, p); break;
      default: launch_factor<18>(grid, nw, st, bd, p); break;
    }
    // one wave per right-hand side, at least four for the staging
    const int waves = (int)std::max<int64_t>(4, std::min<int64_t>(BAND_MC, m));
    hipLaunchKernelGGL(k_band_back, grid, dim3(64 * waves), 0, st, n, bd.kw, mm, p->U, p->Y, p->ustride,
                       p->ystride);
  }
  hipLaunchKernelGGL(k_band_accum, dim3(grid_for(p->n * m)), dim3(256), 0, st, bd.n, bd.m, p->S, p->real, p->w,
                     sh.ec, p->Y, p->ystride, (double2*)X, ldx);
  return hipGetLastError() == hipSuccess ? 0 : EXPM_PFD_ERR_HIP;
}

extern "C" int expm_pfd_band_destroy(expm_pfd_band_t p) {
  if (!p) return EXPM_PFD_ERR_NULL;
  (void)hipDeviceSynchronize();
  band_free(p);
  return 0;
}

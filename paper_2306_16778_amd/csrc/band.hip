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
// pivot magnitude |Re| + |Im|; NaN ranks highest so that it reaches the result
__device__ __forceinline__ double pivot_mag(double2 z) {
  const double m = fabs(z.x) + fabs(z.y);
  return m != m ? INFINITY : m;
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

// A wave's stream over a device array read in chunks of 64 complex values (one
// per lane), two chunks ahead of use, in rising (UP) or falling index order.
// Values come out by readlane (an index shared by the wave) or by a lane shuffle
// (an index per lane); every index asked for lies in the current chunk or the
// next one.
template <bool UP>
struct ChunkStream {
  const double2* p;
  int64_t len, X;  // X: the current chunk
  double2 c0, c1, c2;
  __device__ __forceinline__ double2 ld(int64_t ci, int lane) const {
    const int64_t f = ci * 64 + lane;
    return (ci >= 0 && f < len) ? p[f] : czero<double2>();
  }
  __device__ __forceinline__ void init(const double2* p_, int64_t len_, int64_t first, int lane) {
    constexpr int D = UP ? 1 : -1;
    p = p_;
    len = len_;
    X = first >> 6;
    c0 = ld(X, lane);
    c1 = ld(X + D, lane);
    c2 = ld(X + 2 * D, lane);
  }
  // make the chunk of index f (the lowest index still needed going up, the
  // highest going down) the current one
  __device__ __forceinline__ void reach(int64_t f, int lane) {
    constexpr int D = UP ? 1 : -1;
    const int64_t ci = f >> 6;
    while (UP ? ci > X : ci < X) {
      c0 = c1;
      c1 = c2;
      X += D;
      c2 = ld(X + 2 * D, lane);
    }
  }
  __device__ __forceinline__ double2 uni(int64_t f) const {
    const int l = (int)(f & 63);
    return (f >> 6) == X ? lane_bcast2(c0, l) : lane_bcast2(c1, l);
  }
  __device__ __forceinline__ double2 per(int64_t f) const {
    const int l = (int)(f & 63);
    double2 a, b;
    a.x = __shfl(c0.x, l);
    a.y = __shfl(c0.y, l);
    b.x = __shfl(c1.x, l);
    b.y = __shfl(c1.y, l);
    return (f >> 6) == X ? a : b;
  }
};

// ---- narrow bands: one wave per pole -----------------------------------------
// U: row j of pole k at U + k*ustride + j*(2KD+1): [1/pivot, U(j, j+1), ..., U(j, j+2KD)]
// Y: pole k's n x m solution, row-major (element (j, r) at Y + k*ystride + j*m + r)
template <int KD>
__global__ __launch_bounds__(64) void k_band_narrow(int n, int m, const double2* __restrict__ R,
                                                    const double2* __restrict__ Vr, const double2* __restrict__ pole,
                                                    double2* __restrict__ U, double2* __restrict__ Y,
                                                    int64_t ustride, int64_t ystride) {
  constexpr int W = 2 * KD + 1;
  const int k = blockIdx.x, lane = threadIdx.x;
  const bool act = lane < m;
  const double2 th = pole[k];
  double2* Uk = U + k * ustride;
  double2* Yk = Y + k * ystride;
  ChunkStream<true> rs, vs;  // rows of the matrix, rows of V
  rs.init(R, (int64_t)n * W, 0, lane);
  vs.init(Vr, (int64_t)n * m, 0, lane);
  // row q of tA - cI + theta I at column q - KD + c
  auto row_at = [&](int q, int c) {
    double2 v = q < n ? rs.uni((int64_t)q * W + c) : czero<double2>();
    if (c == KD && q < n) {
      v.x += th.x;
      v.y += th.y;
    }
    return v;
  };
  auto rhs = [&](int q) {
    const double2 v = vs.per((int64_t)q * m + lane);
    return (act && q < n) ? v : czero<double2>();
  };
  double2 w[KD + 1][W], bb[KD + 1];
#pragma unroll
  for (int i = 0; i <= KD; ++i) {
    rs.reach((int64_t)min(i, n - 1) * W, lane);
    vs.reach((int64_t)min(i, n - 1) * m, lane);
#pragma unroll
    for (int c = 0; c < W; ++c) {
      const int off = c - i + KD;  // column c of row i
      w[i][c] = (off >= 0 && off < W) ? row_at(i, off) : czero<double2>();
    }
    bb[i] = rhs(i);
  }
  for (int j = 0; j < n; ++j) {
    const int alive = min(KD + 1, n - j);  // rows of the window that hold matrix rows
    int p = 0;
    double best = pivot_mag(w[0][0]);
#pragma unroll
    for (int i = 1; i <= KD; ++i) {
      const double mg = pivot_mag(w[i][0]);
      if (i < alive && mg > best) {
        best = mg;
        p = i;
      }
    }
#pragma unroll
    for (int i = 1; i <= KD; ++i)
      if (p == i) {
#pragma unroll
        for (int c = 0; c < W; ++c) {
          const double2 x = w[0][c];
          w[0][c] = w[i][c];
          w[i][c] = x;
        }
        const double2 x = bb[0];
        bb[0] = bb[i];
        bb[i] = x;
      }
    const double2 rp = crecip(w[0][0]);
#pragma unroll
    for (int i = 1; i <= KD; ++i) {
      const double2 l = cmul(w[i][0], rp);
#pragma unroll
      for (int c = 1; c < W; ++c) w[i][c] = cfms(w[i][c], l, w[0][c]);
      bb[i] = cfms(bb[i], l, bb[0]);
    }
    if (lane == 0) {
      Uk[(int64_t)j * W] = rp;
#pragma unroll
      for (int c = 1; c < W; ++c) Uk[(int64_t)j * W + c] = w[0][c];
    }
    if (act) Yk[(int64_t)j * m + lane] = bb[0];
    // the window moves one row down and one column right; the new row is matrix
    // row j + KD + 1 over columns j + 1 .. j + 1 + 2KD
#pragma unroll
    for (int i = 0; i < KD; ++i) {
#pragma unroll
      for (int c = 0; c + 1 < W; ++c) w[i][c] = w[i + 1][c + 1];
      w[i][W - 1] = czero<double2>();
      bb[i] = bb[i + 1];
    }
    const int q = j + KD + 1;
    rs.reach((int64_t)min(q, n - 1) * W, lane);
    vs.reach((int64_t)min(q, n - 1) * m, lane);
#pragma unroll
    for (int c = 0; c < W; ++c) w[KD][c] = row_at(q, c);
    bb[KD] = rhs(q);
  }
  __syncthreads();  // U and Y rows written above, read back by other lanes below
  ChunkStream<false> us, ys;
  us.init(Uk, (int64_t)n * W, (int64_t)n * W - 1, lane);
  ys.init(Yk, (int64_t)n * m, (int64_t)n * m - 1, lane);
  double2 xs[2 * KD + 1];  // xs[c - 1] = x_{j + c}
#pragma unroll
  for (int c = 0; c < 2 * KD + 1; ++c) xs[c] = czero<double2>();
  for (int j = n - 1; j >= 0; --j) {
    us.reach((int64_t)j * W + W - 1, lane);
    ys.reach((int64_t)j * m + m - 1, lane);
    double2 s = ys.per((int64_t)j * m + lane);
    if (!act) s = czero<double2>();
#pragma unroll
    for (int c = 1; c < W; ++c) s = cfms(s, us.uni((int64_t)j * W + c), xs[c - 1]);
    const double2 x = cmul(us.uni((int64_t)j * W), s);
#pragma unroll
    for (int c = 2 * KD; c >= 1; --c) xs[c] = xs[c - 1];
    xs[0] = x;
    if (act) Yk[(int64_t)j * m + lane] = x;
  }
}

// LDS-only wait and workgroup barrier: outstanding global loads (the next row)
// and stores (rows of U and Y) stay in flight across it
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt left at their maxima
  __builtin_amdgcn_s_barrier();
}

// ---- wide bands: one workgroup per (pole, block of right-hand sides) ----------
// Same U and Y layouts as the narrow kernel (W = 2 kw + 1); only the first block
// of right-hand sides writes U.
template <int CPW>
__global__ __launch_bounds__(512) void k_band_factor(int n, int kw, int m, const double2* __restrict__ R,
                                                     const double2* __restrict__ Vr,
                                                     const double2* __restrict__ pole, double2* __restrict__ U,
                                                     double2* __restrict__ Y, int64_t ustride, int64_t ystride) {
  __shared__ double2 lbuf[2][64];
  __shared__ int pbuf[2];
  const int k = blockIdx.x, lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int NW = blockDim.x >> 6;
  const int W = 2 * kw + 1;
  const int r0 = blockIdx.y * BAND_MC;
  const int slots = W + min(BAND_MC, m - r0);
  const bool writeU = blockIdx.y == 0;
  const double2 th = pole[k];
  double2* Uk = U + k * ustride;
  double2* Yk = Y + k * ystride;
  // row q of tA - cI + theta I at column q - kw + c
  auto row_at = [&](int q, int c) {
    double2 v = q < n ? R[(int64_t)q * W + c] : czero<double2>();
    if (c == kw && q < n) {
      v.x += th.x;
      v.y += th.y;
    }
    return v;
  };

  double2 a[CPW], pf[CPW];
  bool alive = lane <= kw && lane < n;  // active-row slot `lane` holds matrix row `lane`
  // window at column 0: slot s holds column s; right-hand side slots W + r
#pragma unroll
  for (int i = 0; i < CPW; ++i) {
    const int s = wv + i * NW;
    a[i] = czero<double2>();
    if (alive && s < W) {
      const int off = s - lane + kw;
      if (off >= 0 && off < W) a[i] = row_at(lane, off);
    } else if (alive && s < slots) {
      a[i] = Vr[(int64_t)lane * m + r0 + s - W];
    }
  }
  // the row inserted at the end of step j is row q = j + kw + 1, over the columns
  // of step j + 1: slot s then holds column (j+1) + ((s - (j+1)) mod W), which is
  // entry (s - (j+1)) mod W of the row
  auto prefetch = [&](int j) {
    const int q = j + kw + 1;
    const int s1 = (j + 1) % W;
#pragma unroll
    for (int i = 0; i < CPW; ++i) {
      const int s = wv + i * NW;
      pf[i] = czero<double2>();
      if (q < n && s < W) pf[i] = row_at(q, s >= s1 ? s - s1 : s - s1 + W);
      else if (q < n && s < slots) pf[i] = Vr[(int64_t)q * m + r0 + s - W];
    }
  };
  // pivot and multipliers of column j, held in z (run by the wave holding it)
  auto pivot = [&](double2 z, int nb, int j) {
    double mg = alive ? pivot_mag(z) : -1.0;
    const double mx = wave_max(mg);
    int pl = wave_min(mg == mx ? lane : 64);
    if (pl >= 64) pl = 0;  // (mx is one of the lanes' values)
    const double2 piv = lane_bcast2(z, pl);
    const double2 rp = crecip(piv);
    lbuf[nb][lane] = (alive && lane != pl) ? cmul(z, rp) : czero<double2>();
    if (lane == 0) {
      pbuf[nb] = pl;
      if (writeU) Uk[(int64_t)j * W] = rp;
    }
  };
  prefetch(0);
#pragma unroll
  for (int i = 0; i < CPW; ++i)
    if (wv + i * NW == 0) pivot(a[i], 0, 0);
  lds_barrier();
  for (int j = 0; j < n; ++j) {
    const int buf = j & 1;
    const int p = __builtin_amdgcn_readfirstlane(pbuf[buf]);
    const double2 l = lbuf[buf][lane];
    const bool qin = j + kw + 1 < n;
    const int sj = j % W;  // slot of column j: it leaves, and takes column j + W
#pragma unroll
    for (int i = 0; i < CPW; ++i) {
      const int s = wv + i * NW;
      if (s >= slots) continue;
      const double2 pv = lane_bcast2(a[i], p);
      if (s < W) {
        const int cofs = s >= sj ? s - sj : s - sj + W;  // column - j
        if (lane == p) {
          if (writeU && cofs > 0) Uk[(int64_t)j * W + cofs] = a[i];
          a[i] = pf[i];
        } else {
          // column j + W is zero in the remaining rows (they end before it)
          a[i] = cofs == 0 ? czero<double2>() : cfms(a[i], l, pv);
        }
      } else {
        if (lane == p) {
          Yk[(int64_t)j * m + r0 + s - W] = a[i];
          a[i] = pf[i];
        } else {
          a[i] = cfms(a[i], l, pv);
        }
      }
    }
    if (lane == p) alive = qin;
    if (j + 1 < n) {
      prefetch(j + 1);
      const int s1 = (j + 1) % W;
#pragma unroll
      for (int i = 0; i < CPW; ++i)
        if (wv + i * NW == s1) pivot(a[i], buf ^ 1, j + 1);
    }
    lds_barrier();
  }
}

// back substitution x_j = (1/u_jj) (y_j - sum_{c=1..2kw} u_{j,j+c} x_{j+c}), in place
// in Y; one wave per right-hand side.  Each lane's two coefficients, the pivot's
// reciprocal and y_j are loaded BACK_AHEAD rows ahead (a register queue, the
// loop unrolled by its length).
constexpr int BACK_AHEAD = 4;
__global__ __launch_bounds__(1024) void k_band_back(int n, int kw, int m, const double2* __restrict__ U,
                                                    double2* __restrict__ Y, int64_t ustride, int64_t ystride) {
  const int k = blockIdx.x, lane = threadIdx.x & 63;
  const int r = blockIdx.y * BAND_MC + (threadIdx.x >> 6);
  if (r >= m) return;
  const int W = 2 * kw + 1;
  const double2* Uk = U + k * ustride;
  double2* Yk = Y + k * ystride;
  // ring: x_i at position i mod 128, positions lane and lane + 64
  double2 x0 = czero<double2>(), x1 = czero<double2>();
  struct Row {
    double2 u0, u1, rp, y;
  };
  auto load = [&](int j) {
    Row q;
    q.u0 = q.u1 = q.rp = q.y = czero<double2>();
    if (j >= 0) {
      const int c0 = (lane - j) & 127, c1 = (lane + 64 - j) & 127;
      if (c0 >= 1 && c0 < W && j + c0 < n) q.u0 = Uk[(int64_t)j * W + c0];
      if (c1 >= 1 && c1 < W && j + c1 < n) q.u1 = Uk[(int64_t)j * W + c1];
      q.rp = Uk[(int64_t)j * W];
      q.y = Yk[(int64_t)j * m + r];
    }
    return q;
  };
  auto step = [&](int j, const Row& q) {
    double2 t = cmul(q.u0, x0);
    t.x += q.u1.x * x1.x - q.u1.y * x1.y;
    t.y += q.u1.x * x1.y + q.u1.y * x1.x;
    double2 s;
    s.x = q.y.x - wave_sum_dpp(t.x);
    s.y = q.y.y - wave_sum_dpp(t.y);
    const double2 x = cmul(q.rp, s);
    if ((j & 63) == lane) {
      if (j & 64) x1 = x;
      else x0 = x;
    }
    if (lane == 0) Yk[(int64_t)j * m + r] = x;
  };
  Row qu[BACK_AHEAD];
#pragma unroll
  for (int i = 0; i < BACK_AHEAD; ++i) qu[i] = load(n - 1 - i);
  for (int j0 = n - 1; j0 >= 0; j0 -= BACK_AHEAD) {
#pragma unroll
    for (int i = 0; i < BACK_AHEAD; ++i) {
      const int j = j0 - i;
      if (j >= 0) {
        step(j, qu[i]);
        qu[i] = load(j - BACK_AHEAD);
      }
    }
  }
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
};

namespace {
void band_free(expm_pfd_band_t p) {
  if (!p) return;
  void* ptrs[] = {p->pole, p->w, p->U, p->Y, p->R, p->Vr};
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
  p->ustride = n * W;
  p->ystride = n * m_max;
  bool ok = hipMalloc((void**)&p->pole, p->S * sizeof(double2)) == hipSuccess &&
            hipMalloc((void**)&p->w, p->S * sizeof(double2)) == hipSuccess &&
            hipMalloc((void**)&p->U, (size_t)p->S * p->ustride * sizeof(double2)) == hipSuccess &&
            hipMalloc((void**)&p->Y, (size_t)p->S * p->ystride * sizeof(double2)) == hipSuccess &&
            hipMalloc((void**)&p->R, (size_t)n * W * sizeof(double2)) == hipSuccess &&
            hipMalloc((void**)&p->Vr, (size_t)n * m_max * sizeof(double2)) == hipSuccess;
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
  const dim3 g1((unsigned)p->S);
  const int n = bd.n, mm = bd.m;
  if (p->kw <= BAND_NARROW_KD) {
#define EXPM_BAND_NARROW(KD) \
  hipLaunchKernelGGL(k_band_narrow<KD>, g1, dim3(64), 0, st, n, mm, p->R, p->Vr, p->pole, p->U, p->Y, p->ustride, \
                     p->ystride)
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
    const int nw = (slots + cpw - 1) / cpw;
    const dim3 grid((unsigned)p->S, (unsigned)chunks);
    switch (cpw) {
      case 2: launch_factor<2>(grid, nw, st, bd, p); break;
      case 4: launch_factor<4>(grid, nw, st, bd, p); break;
      case 8: launch_factor<8>(grid, nw, st, bd, p); break;
      case 12: launch_factor<12>(grid, nw, st, bd, p); break;
      default: launch_factor<18>(grid, nw, st, bd, p); break;
    }
    const int waves = (int)std::min<int64_t>(BAND_MC, m);
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

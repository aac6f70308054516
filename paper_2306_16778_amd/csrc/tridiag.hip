// libexpm_pfd, tridiagonal route: exp(tA)V ~ R_d(tA)V for several t from one
// reduction of A (see include/expm_pfd.h, expm_pfd_tridiag_*).
//
// The paper notes that its partial-fraction form combines with a reduction of A
// to tridiagonal form (Sec. 1): with A = Q T Q^H, T real symmetric tridiagonal
// and Q unitary,
//   R_d(tA) V = Q [ sum_k a_k (tT + theta_k I)^{-1} ] Q^H V,
// so the O(n^3) work is done once per matrix and every later t costs two
// products with Q (O(n^2 m)) and d/2 tridiagonal solves per column (O(n)).
//
// factor:  Householder reduction of the Hermitian A, one column at a time: the
//   reflector of column j is generated from row j (the conjugate of the column
//   below the diagonal; every update keeps the full matrix Hermitian), then
//   y = A22 v (one kernel), and A22 -= v w^H + w v^H with w = tau y - c v,
//   c = |tau|^2 (y^H v) / 2 (one kernel, which also generates the next reflector
//   from the row it has just updated).  The reflectors are kept below the
//   diagonal; Q is then formed explicitly, 32 reflectors at a time in compact
//   WY form on the matrix cores.
// apply:   B = Q^H V; per pole pair one LU factorization with partial pivoting
//   of the tridiagonal tT + theta I (one thread per pole), then solves for B and
//   for conj(B) (the conjugate pole: T is real, so (tT + conj(theta) I)^{-1} b =
//   conj((tT + theta I)^{-1} conj(b))), one thread per right-hand side; the
//   residue-weighted sum in FP64; X = Q Z.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "host_common.h"
#include "kernels.h"
#include "spike.h"

using namespace expm;

namespace {

constexpr int TRI_NB = 32;       // reflectors per compact-WY block of the Q formation
constexpr int TRI_KS = 16;       // most K slices of the Q formation's reductions over the rows
constexpr int TRI_PAD = 256;     // zero rows past the n of Q and of the reflector panel (slice padding)
constexpr int ROWS_PER_WG = 4;  // rows per workgroup of the reduction kernels (one per wave)
constexpr int FUSED_ROWS = 8;   // rows per workgroup of the fused reduction step (one per wave)
constexpr int FUSED_NT = 64 * FUSED_ROWS;

// ---- wave reductions ----------------------------------------------------------
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
  return x;
}
__device__ __forceinline__ double2 wave_sum2(double2 x) {
  x.x = wave_sum(x.x);
  x.y = wave_sum(x.y);
  return x;
}

// Householder reflector H = I - tau v v^H with H^H x = beta e_1, beta real, for
// x_r = conj(A[j][r]), r = j+1 .. n-1 (column j below the diagonal of the
// Hermitian matrix, read along row j).  Run by one whole wave.  v (v_0 = 1) goes
// to vbuf[0 .. L) and below the diagonal of column j (A[r][j], r > j); tau, the
// subdiagonal beta and the diagonal Re A[j][j] to tau[j], e[j], d[j].
__device__ void householder_from_row(double2* __restrict__ A, int64_t ld, int n, int j, double2* __restrict__ vbuf,
                                     double2* __restrict__ tau, double* __restrict__ e, double* __restrict__ d) {
  const int lane = threadIdx.x & 63;
  const double2* row = A + (int64_t)j * ld;
  const int L = n - j - 1;
  double sig = 0.0;
  for (int r = j + 2 + lane; r < n; r += 64) {
    const double2 x = row[r];
    sig += x.x * x.x + x.y * x.y;
  }
  sig = wave_sum(sig);
  const double2 alpha = cconj(row[j + 1]);
  double2 t, s;
  double beta;
  if (sig == 0.0 && alpha.y == 0.0) {
    t = czero<double2>();
    beta = alpha.x;
    s = czero<double2>();
  } else {
    const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + sig);
    beta = alpha.x >= 0.0 ? -nrm : nrm;
    t.x = (beta - alpha.x) / beta;
    t.y = -alpha.y / beta;
    double2 am;  // alpha - beta
    am.x = alpha.x - beta;
    am.y = alpha.y;
    s = crecip(am);
  }
  for (int r = j + 1 + lane; r < n; r += 64) {
    double2 v;
    if (r == j + 1) {
      v.x = 1.0;
      v.y = 0.0;
    } else {
      v = cmul(cconj(row[r]), s);
    }
    vbuf[r - j - 1] = v;
    A[(int64_t)r * ld + j] = v;
  }
  if (lane == 0) {
    tau[j] = t;
    e[j] = beta;
    d[j] = row[j].x;
  }
  (void)L;
}

// The first reflector (column 0).  grid 1, block 64
__global__ __launch_bounds__(64) void k_tri_house0(double2* __restrict__ A, int64_t ld, int n,
                                                   double2* __restrict__ vbuf, double2* __restrict__ tau,
                                                   double* __restrict__ e, double* __restrict__ d) {
  householder_from_row(A, ld, n, 0, vbuf, tau, e, d);
}

// Coherent read of a double2 written by another workgroup of the same launch
// (two agent-scope atomic loads: no stale line of this CU's cache is used).
__device__ __forceinline__ double2 load_coherent(const double2* p) {
  const unsigned long long* q = (const unsigned long long*)p;
  double2 r;
  r.x = __longlong_as_double((long long)__hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  r.y = __longlong_as_double((long long)__hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  return r;
}

// y = A22 v for step j (A22 = rows and columns j+1 .. n-1 of A, v in vbuf), one
// row per wave, four independent partial sums per lane.  The workgroups' sums of
// conj(y_r) v_r go to part[], and the last workgroup to finish (counted in
// *done) adds them in a fixed order into *yv and clears *done.
// grid ceil(L / ROWS_PER_WG), block 256
__global__ __launch_bounds__(256) void k_tri_gemv(const double2* __restrict__ A, int64_t ld, int n, int j,
                                                  const double2* __restrict__ vbuf, double2* __restrict__ y,
                                                  double2* __restrict__ part, double2* __restrict__ yv,
                                                  unsigned* __restrict__ done) {
  __shared__ double2 red[256];
  __shared__ bool last;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int L = n - j - 1;
  const int i = blockIdx.x * ROWS_PER_WG + wave;  // row j+1+i of A
  double2 acc = czero<double2>();
  if (i < L) {
    const double2* row = A + (int64_t)(j + 1 + i) * ld + (j + 1);
    double2 s[4] = {czero<double2>(), czero<double2>(), czero<double2>(), czero<double2>()};
    int c = lane;
    for (; c + 192 < L; c += 256) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double2 a = row[c + 64 * u], v = vbuf[c + 64 * u];
        s[u].x += a.x * v.x - a.y * v.y;
        s[u].y += a.x * v.y + a.y * v.x;
      }
    }
    for (; c < L; c += 64) {
      const double2 a = row[c], v = vbuf[c];
      s[0].x += a.x * v.x - a.y * v.y;
      s[0].y += a.x * v.y + a.y * v.x;
    }
    double2 t;
    t.x = (s[0].x + s[1].x) + (s[2].x + s[3].x);
    t.y = (s[0].y + s[1].y) + (s[2].y + s[3].y);
    t = wave_sum2(t);
    if (lane == 0) {
      y[i] = t;
      const double2 v = vbuf[i];
      acc.x = t.x * v.x + t.y * v.y;  // conj(y_i) v_i
      acc.y = t.x * v.y - t.y * v.x;
    }
  }
  if (lane == 0) red[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 w = red[0];
    for (int k = 1; k < 4; ++k) {
      w.x += red[k].x;
      w.y += red[k].y;
    }
    part[blockIdx.x] = w;
    __threadfence();
    last = atomicAdd(done, 1u) == gridDim.x - 1u;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double2 t = czero<double2>();
  for (unsigned b = threadIdx.x; b < gridDim.x; b += 256) {
    const double2 p = load_coherent(part + b);
    t.x += p.x;
    t.y += p.y;
  }
  red[threadIdx.x] = t;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) {
      red[threadIdx.x].x += red[threadIdx.x + h].x;
      red[threadIdx.x].y += red[threadIdx.x + h].y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *yv = red[0];
    *done = 0u;
  }
}

// A22 -= v w^H + w v^H for step j with w = tau y - c v, c = |tau|^2 Re(y^H v) / 2,
// one row per wave (row j+1 .. n-1).  Below the diagonal, column j+1 is left as
// it is (no later step reads it; it receives the next reflector).  The wave that
// updates row j+1 then generates the reflector of column j+1 from it (into the
// other half of the reflector buffer), or, for the last row, records d[n-1].
// grid ceil(L / ROWS_PER_WG), block 256
__global__ __launch_bounds__(256) void k_tri_update(double2* __restrict__ A, int64_t ld, int n, int j,
                                                    const double2* __restrict__ vbuf, double2* __restrict__ vnext,
                                                    const double2* __restrict__ y, const double2* __restrict__ yv,
                                                    double2* __restrict__ tau, double* __restrict__ e,
                                                    double* __restrict__ d) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int L = n - j - 1;
  const double2 t = tau[j];
  const double cc = 0.5 * (t.x * t.x + t.y * t.y) * yv->x;
  const int i = blockIdx.x * ROWS_PER_WG + wave;
  if (i < L) {
    double2* row = A + (int64_t)(j + 1 + i) * ld + (j + 1);
    const double2 vi = vbuf[i], yi = y[i];
    double2 wi = cmul(t, yi);
    wi.x -= cc * vi.x;
    wi.y -= cc * vi.y;
    for (int c = (i == 0 ? 0 : 1) + lane; c < L; c += 64) {
      const double2 vc = vbuf[c];
      double2 wc = cmul(t, y[c]);
      wc.x -= cc * vc.x;
      wc.y -= cc * vc.y;
      // a -= v_i conj(w_c) + w_i conj(v_c)
      double2 a = row[c];
      a.x -= vi.x * wc.x + vi.y * wc.y + wi.x * vc.x + wi.y * vc.y;
      a.y -= vi.y * wc.x - vi.x * wc.y + wi.y * vc.x - wi.x * vc.y;
      row[c] = a;
    }
  }
  if (blockIdx.x == 0 && wave == 0) {
    __threadfence_block();  // the row's updated entries, stored by other lanes, are read next
    if (j + 1 <= n - 2) {
      householder_from_row(A, ld, n, j + 1, vnext, tau, e, d);
    } else if (lane == 0) {
      d[n - 1] = A[(int64_t)(n - 1) * ld + (n - 1)].x;
    }
  }
}

// Step j's rank-2 update fused with step j+1's product y' = A22' v' (one pass
// over the trailing matrix per step instead of two).  Every workgroup first
// forms row j+1 after step j's update (in LDS) and, from it, the reflector v' of
// step j+1 exactly as householder_from_row does (the same arithmetic and the
// same reduction order in every workgroup, so all copies have the same bits);
// workgroup 0 stores v' (below the diagonal of column j+1 and into vnext) and
// tau, e, d of step j+1.  Each wave then updates its rows j+2 .. n-1 (columns
// j+2 .. n-1; column j+1 is left as it is, it holds the reflector) and forms
// y'_k from the values it has just stored.  Row j+1 itself is not stored: no
// later step reads it.  The workgroups' sums of conj(y'_k) v'_k go to part[],
// and the last workgroup to finish adds them in a fixed order into *yvnext and
// clears *done.
// grid ceil((L - 1) / FUSED_ROWS) with L = n - j - 1 >= 2, block FUSED_NT (one
// row per wave), dynamic LDS L x 16 bytes
__global__ __launch_bounds__(FUSED_NT) void k_tri_step(double2* __restrict__ A, int64_t ld, int n, int j,
                                                       const double2* __restrict__ v, double2* __restrict__ vnext,
                                                       const double2* __restrict__ y, double2* __restrict__ ynext,
                                                       const double2* __restrict__ yv, double2* __restrict__ yvnext,
                                                       double2* __restrict__ tau, double* __restrict__ e,
                                                       double* __restrict__ d, double2* __restrict__ part,
                                                       unsigned* __restrict__ done) {
  extern __shared__ double2 rowb[];  // row j+1 after the update, then v' (entry c: column j+1+c)
  __shared__ double red[FUSED_ROWS];
  __shared__ double2 red2[FUSED_NT];
  __shared__ bool last;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int L = n - j - 1;
  const double2 t = tau[j];
  const double cc = 0.5 * (t.x * t.x + t.y * t.y) * yv->x;
  // w_c = tau y_c - cc v_c, as in k_tri_update
  auto wof = [&](int c, double2 vc) {
    double2 w = cmul(t, y[c]);
    w.x -= cc * vc.x;
    w.y -= cc * vc.y;
    return w;
  };
  {
    // four columns per pass, their loads issued together
    const double2 v0 = v[0], w0 = wof(0, v0);
    const double2* row1 = A + (int64_t)(j + 1) * ld + (j + 1);
    for (int c0 = tid; c0 < L; c0 += 4 * FUSED_NT) {
      double2 av[4], vv[4], yy[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = c0 + FUSED_NT * u < L ? c0 + FUSED_NT * u : c0;
        av[u] = row1[c];
        vv[u] = v[c];
        yy[u] = y[c];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = c0 + FUSED_NT * u;
        if (c < L) {
          const double2 vc = vv[u];
          double2 wc = cmul(t, yy[u]);
          wc.x -= cc * vc.x;
          wc.y -= cc * vc.y;
          double2 a = av[u];
          a.x -= v0.x * wc.x + v0.y * wc.y + w0.x * vc.x + w0.y * vc.y;
          a.y -= v0.y * wc.x - v0.x * wc.y + w0.y * vc.x - w0.x * vc.y;
          rowb[c] = a;
        }
      }
    }
  }
  __syncthreads();
  // the reflector of step j+1 from x_c = conj(rowb[c]), c = 1 .. L-1
  double sig = 0.0;
  for (int c = 2 + tid; c < L; c += FUSED_NT) {
    const double2 x = rowb[c];
    sig += x.x * x.x + x.y * x.y;
  }
  sig = wave_sum(sig);
  if (lane == 0) red[wave] = sig;
  __syncthreads();
  sig = 0.0;
#pragma unroll
  for (int w = 0; w < FUSED_ROWS; ++w) sig += red[w];
  const double2 alpha = cconj(rowb[1]);
  const double dnext = rowb[0].x;
  double2 tn, sc;
  double beta;
  if (sig == 0.0 && alpha.y == 0.0) {
    tn = czero<double2>();
    beta = alpha.x;
    sc = czero<double2>();
  } else {
    const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + sig);
    beta = alpha.x >= 0.0 ? -nrm : nrm;
    tn.x = (beta - alpha.x) / beta;
    tn.y = -alpha.y / beta;
    double2 am;  // alpha - beta
    am.x = alpha.x - beta;
    am.y = alpha.y;
    sc = crecip(am);
  }
  __syncthreads();  // rowb[0] and rowb[1] have been read everywhere
  for (int c = 1 + tid; c < L; c += FUSED_NT) {
    double2 vv;
    if (c == 1) {
      vv.x = 1.0;
      vv.y = 0.0;
    } else {
      vv = cmul(cconj(rowb[c]), sc);
    }
    rowb[c] = vv;
    if (blockIdx.x == 0) {
      A[(int64_t)(j + 1 + c) * ld + (j + 1)] = vv;
      vnext[c - 1] = vv;
    }
  }
  if (blockIdx.x == 0 && tid == 0) {
    tau[j + 1] = tn;
    e[j + 1] = beta;
    d[j + 1] = dnext;
  }
  __syncthreads();
  // rows j+2 .. n-1: row j+1+i with i = k + 1, k = blockIdx.x * FUSED_ROWS + wave
  double2 acc = czero<double2>();
  {
    const int k = blockIdx.x * FUSED_ROWS + wave;
    if (k < L - 1) {
      const int i = k + 1;
      double2* row = A + (int64_t)(j + 1 + i) * ld + (j + 1);
      const double2 vi = v[i], wi = wof(i, vi);
      // four columns per pass (their loads issued together), four partial sums
      double2 s4[4] = {czero<double2>(), czero<double2>(), czero<double2>(), czero<double2>()};
      for (int c0 = 1 + lane; c0 < L; c0 += 256) {
        double2 av[4], vv[4], yy[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = c0 + 64 * u < L ? c0 + 64 * u : c0;
          av[u] = row[c];
          vv[u] = v[c];
          yy[u] = y[c];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = c0 + 64 * u;
          if (c < L) {
            const double2 vc = vv[u];
            double2 wc = cmul(t, yy[u]);
            wc.x -= cc * vc.x;
            wc.y -= cc * vc.y;
            double2 a = av[u];
            a.x -= vi.x * wc.x + vi.y * wc.y + wi.x * vc.x + wi.y * vc.y;
            a.y -= vi.y * wc.x - vi.x * wc.y + wi.y * vc.x - wi.x * vc.y;
            row[c] = a;
            const double2 vn = rowb[c];  // v'_{c-1}
            s4[u].x += a.x * vn.x - a.y * vn.y;
            s4[u].y += a.x * vn.y + a.y * vn.x;
          }
        }
      }
      double2 sum;
      sum.x = (s4[0].x + s4[1].x) + (s4[2].x + s4[3].x);
      sum.y = (s4[0].y + s4[1].y) + (s4[2].y + s4[3].y);
      sum = wave_sum2(sum);
      if (lane == 0) {
        ynext[k] = sum;
        const double2 vk = rowb[k + 1];  // v'_k
        acc.x += sum.x * vk.x + sum.y * vk.y;  // conj(y'_k) v'_k
        acc.y += sum.x * vk.y - sum.y * vk.x;
      }
    }
  }
  if (lane == 0) red2[wave] = acc;
  __syncthreads();
  if (tid == 0) {
    double2 w = red2[0];
    for (int k = 1; k < FUSED_ROWS; ++k) {
      w.x += red2[k].x;
      w.y += red2[k].y;
    }
    part[blockIdx.x] = w;
    __threadfence();
    last = atomicAdd(done, 1u) == gridDim.x - 1u;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  double2 q = czero<double2>();
  for (unsigned b = tid; b < gridDim.x; b += FUSED_NT) {
    const double2 pb = load_coherent(part + b);
    q.x += pb.x;
    q.y += pb.y;
  }
  red2[tid] = q;
  __syncthreads();
  for (int h = FUSED_NT / 2; h >= 1; h >>= 1) {
    if (tid < h) {
      red2[tid].x += red2[tid + h].x;
      red2[tid].y += red2[tid + h].y;
    }
    __syncthreads();
  }
  if (tid == 0) {
    *yvnext = red2[0];
    *done = 0u;
  }
}

// d[0] = Re A[0][0] for a matrix of order 1 (no reflector).  grid 1, block 1
__global__ void k_tri_order1(const double2* __restrict__ A, double* __restrict__ d) { d[0] = A[0].x; }

// The reflectors j0 .. j0+nb-1 as a clean L x nb panel (rows j0+1 .. n-1 of A
// below the diagonal, zeros above each reflector's leading 1), row-major.
// grid-stride over L*nb
__global__ __launch_bounds__(256) void k_tri_vpanel(const double2* __restrict__ A, int64_t ld, int n, int j0, int nb,
                                                    int Lpad, double2* __restrict__ Vp) {
  const int L = n - j0 - 1;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)Lpad * nb;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / nb), k = (int)(e % nb);
    // row j0+1+r, reflector j0+k: nonzero from row j0+k+1 on; rows past L are the
    // zero padding of the K slices
    Vp[e] = (r >= k && r < L) ? A[(int64_t)(j0 + 1 + r) * ld + j0 + k] : czero<double2>();
  }
}

// out[e] = sum_{s < ks} part[s * stride + e] in slice order (the K slices of a
// product).  grid-stride over count
__global__ __launch_bounds__(256) void k_tri_sum_slices(const double2* __restrict__ part, int ks, int64_t stride,
                                                        int64_t count, double2* __restrict__ out) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
    double2 acc = part[e];
    for (int s = 1; s < ks; ++s) {
      const double2 p = part[s * stride + e];
      acc.x += p.x;
      acc.y += p.y;
    }
    out[e] = acc;
  }
}

// Triangular factor of the compact WY form H_0 H_1 ... H_{nb-1} = I - V T V^H:
// T upper triangular, T_aa = tau_a, T[a][i] = -tau_i sum_{b=a}^{i-1} T[a][b] S[b][i]
// (S = V^H V, nb x nb, row-major, from a product).  Row a depends only on its own
// earlier entries, so each thread computes one row.
// grid 1, block 64
__global__ __launch_bounds__(64) void k_tri_tfactor(const double2* __restrict__ S, int nb,
                                                    const double2* __restrict__ tau, double2* __restrict__ T) {
  __shared__ double2 Ss[TRI_NB][TRI_NB + 1];
  __shared__ double2 Ts[TRI_NB][TRI_NB + 1];  // row a belongs to thread a
  for (int q = threadIdx.x; q < nb * nb; q += blockDim.x) Ss[q / nb][q % nb] = S[q];
  __syncthreads();
  const int a = threadIdx.x;
  if (a >= nb) return;
  double2* row = Ts[a];
  for (int i = 0; i < nb; ++i) row[i] = czero<double2>();
  row[a] = tau[a];
  for (int i = a + 1; i < nb; ++i) {
    double2 s = czero<double2>();
    for (int b = a; b < i; ++b) {
      const double2 m = cmul(row[b], Ss[b][i]);
      s.x += m.x;
      s.y += m.y;
    }
    const double2 v = cmul(tau[i], s);
    row[i].x = -v.x;
    row[i].y = -v.y;
  }
  for (int i = 0; i < nb; ++i) T[a * nb + i] = row[i];
}

// Q (rows x ld, row-major) = the identity in its n x n leading block, zero elsewhere.
// grid-stride
__global__ __launch_bounds__(256) void k_tri_eye(double2* __restrict__ Q, int64_t ld, int rows, int n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)rows * ld;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / ld, c = e % ld;
    double2 v = czero<double2>();
    if (r == c && r < n) v.x = 1.0;
    Q[e] = v;
  }
}

// Column-major n x m (ld) into row-major n x m, or back (to_col).  grid-stride
__global__ __launch_bounds__(256) void k_tri_layout(const double2* __restrict__ src, int64_t lds,
                                                    double2* __restrict__ dst, int64_t ldd, int n, int m, int to_col) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)n * m;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (to_col) {
      const int r = (int)(e % n), c = (int)(e / n);  // consecutive threads: consecutive rows of a column
      dst[r + (int64_t)c * ldd] = src[(int64_t)r * lds + c];
    } else {
      const int r = (int)(e % n), c = (int)(e / n);
      dst[(int64_t)r * ldd + c] = src[r + (int64_t)c * lds];
    }
  }
}

// One pole per wave (or two waves when 2m > 64): every lane factors the pole's
// tridiagonal matrix t T + (theta_p - c) I by Gaussian elimination with partial
// pivoting (the pivot of column i is the carried row or the original row i+1,
// whichever is larger in |Re| + |Im|, the carried row on ties; the factor is
// the same in every lane), and carries its own right-hand side: column q of B
// (row-major n x m) for lane q < m, its conjugate for m <= q < 2m.  Row i of the
// upper factor (reciprocal pivot, two superdiagonals) is uniform across the
// wave: lane i mod 16 keeps it and lanes 0..15 store 16 rows at once (F, row-
// major per pole); the eliminated right-hand sides go to Ub[row][thread].  The
// back substitution reads 16 rows of factors at once (one per lane) and takes
// each row from its lane by readlane.  Thread index of right-hand side q of
// pole p: p * 2m + q.
// grid (P, ceil(2m / 64)), block 64
constexpr int SOLVE_CHUNK = 16;

__global__ __launch_bounds__(64) void k_tri_solve(const double* __restrict__ d, const double* __restrict__ e, int n,
                                                  double t, const double2* __restrict__ theta, int P, double c,
                                                  const double2* __restrict__ B, int m, double2* __restrict__ F,
                                                  double2* __restrict__ Ub, double2* __restrict__ Y) {
  const int p = blockIdx.x, lane = threadIdx.x;
  const int q = blockIdx.y * 64 + lane;
  const int nt = P * 2 * m;
  const bool act = q < 2 * m;
  const int id = p * 2 * m + q;
  const bool cj = q >= m;
  const int col = act ? (cj ? q - m : q) : 0;
  // factors of pole p, this workgroup's own copy: 3 complex per row (the third:
  // the real second superdiagonal)
  double2* Fp = F + ((int64_t)p * gridDim.y + blockIdx.y) * n * 3;
  double2 sh = theta[p];
  sh.x -= c;
  auto mag = [](double2 z) { return fabs(z.x) + fabs(z.y); };
  auto rhs = [&](int i) {
    double2 b = B[(int64_t)i * m + col];
    if (cj) b.y = -b.y;
    return b;
  };
  double2 cp, cq, cb;
  cp.x = t * d[0] + sh.x;
  cp.y = sh.y;
  cq.x = n > 1 ? t * e[0] : 0.0;
  cq.y = 0.0;
  cb = rhs(0);
  double2 kr = czero<double2>(), k1 = czero<double2>();  // this lane's kept row: 1/u_ii, u_i,i+1
  double k2 = 0.0;                                       // u_i,i+2
  for (int i0 = 0; i0 + 1 < n; i0 += SOLVE_CHUNK) {
    double dn_[SOLVE_CHUNK], off_[SOLVE_CHUNK + 1];
    double2 bn_[SOLVE_CHUNK];
#pragma unroll
    for (int k = 0; k < SOLVE_CHUNK; ++k) {
      const bool in = i0 + k + 1 < n;
      dn_[k] = in ? d[i0 + k + 1] : 0.0;
      off_[k] = in ? e[i0 + k] : 0.0;
      bn_[k] = in ? rhs(i0 + k + 1) : czero<double2>();
    }
    off_[SOLVE_CHUNK] = i0 + SOLVE_CHUNK + 1 < n ? e[i0 + SOLVE_CHUNK] : 0.0;
#pragma unroll
    for (int k = 0; k < SOLVE_CHUNK; ++k) {
      const int i = i0 + k;
      // (predicated, not left early: the chunk's arrays must stay in registers)
      if (i + 1 < n) {
        const double off = t * off_[k];  // A[i+1][i] = A[i][i+1]
        double2 dn;                      // A[i+1][i+1]
        dn.x = t * dn_[k] + sh.x;
        dn.y = sh.y;
        const double offn = i + 2 < n ? t * off_[k + 1] : 0.0;  // A[i+1][i+2]
        // without interchange U row i is the carry (cp, cq, 0) and row i+1 loses
        // l times it; with one, U row i is the original row i+1 (off, dn, offn)
        // and the carry loses l times that
        const bool sw = !(mag(cp) >= fabs(off));
        double2 piv = cp, oth;
        oth.x = off;
        oth.y = 0.0;
        if (sw) {
          piv = oth;
          oth = cp;
        }
        const double2 r = crecip_fast(piv);
        const double2 l = cmul(oth, r);
        const double2 u1 = sw ? dn : cq;
        const double2 keep = sw ? cq : dn;  // carry' = keep - l * u1
        if (lane == k) {
          kr = r;
          k1 = u1;
          k2 = sw ? offn : 0.0;
        }
        const double2 ub = sw ? bn_[k] : cb;
        cb = sw ? cfms(cb, l, bn_[k]) : cfms(bn_[k], l, cb);
        if (act) Ub[(int64_t)i * nt + id] = ub;
        cp = cfms(keep, l, u1);
        cq.x = sw ? -l.x * offn : offn;
        cq.y = sw ? -l.y * offn : 0.0;
      }
    }
    // rows i0 .. i0+15 of the factor, one per lane
    if (lane < SOLVE_CHUNK && i0 + lane + 1 < n) {
      double2* Fi = Fp + (int64_t)(i0 + lane) * 3;
      Fi[0] = kr;
      Fi[1] = k1;
      Fi[2] = double2{k2, 0.0};
    }
  }
  const double2 rl = crecip_fast(cp);  // last pivot
  double2 x1 = cmul(cb, rl);
  if (act) Y[(int64_t)(n - 1) * nt + id] = x1;
  double2 x2 = czero<double2>();
  // the factor rows were stored by other lanes of this wave
  __threadfence_block();
  for (int top = n - 2; top >= 0; top -= SOLVE_CHUNK) {
    // lane k < 16 holds row top - k of the factor; every lane its 16 eliminated rhs
    double2 fr = czero<double2>(), f1 = czero<double2>();
    double f2 = 0.0;
    if (lane < SOLVE_CHUNK && top - lane >= 0) {
      const double2* Fi = Fp + (int64_t)(top - lane) * 3;
      fr = Fi[0];
      f1 = Fi[1];
      f2 = Fi[2].x;
    }
    double2 ub_[SOLVE_CHUNK];
#pragma unroll
    for (int k = 0; k < SOLVE_CHUNK; ++k) {
      const int i = top - k;
      ub_[k] = (i >= 0 && act) ? Ub[(int64_t)i * nt + id] : czero<double2>();
    }
#pragma unroll
    for (int k = 0; k < SOLVE_CHUNK; ++k) {
      const int i = top - k;
      if (i >= 0) {
        const double2 r = lane_bcast2(fr, k), u1 = lane_bcast2(f1, k);
        const double u2 = lane_bcast(f2, k);
        double2 v = cfms(ub_[k], u1, x1);
        v.x -= u2 * x2.x;
        v.y -= u2 * x2.y;
        const double2 x = cmul(v, r);
        if (act) Y[(int64_t)i * nt + id] = x;
        x2 = x1;
        x1 = x;
      }
    }
  }
}

// Z[r][q] = sum_p (e^c a_p Y[r][p, q] + conj(e^c a_p Y[r][p, m+q])) in the fixed
// pair order (Y as written by k_tri_solve).  grid-stride over n*m
__global__ __launch_bounds__(256) void k_tri_accum(const double2* __restrict__ Y, int n, int m, int P,
                                                   const double2* __restrict__ a, double ec,
                                                   double2* __restrict__ Z) {
  const int nt = P * 2 * m;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)n * m;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(e / m), q = (int)(e % m);
    const double2* row = Y + (int64_t)r * nt;
    double sr = 0.0, si = 0.0;
    for (int p = 0; p < P; ++p) {
      double2 ap = a[p];
      ap.x *= ec;
      ap.y *= ec;
      const double2 y = row[p * 2 * m + q], z = row[p * 2 * m + m + q];
      // a y + conj(a z)
      sr += ap.x * y.x - ap.y * y.y + ap.x * z.x - ap.y * z.y;
      si += ap.x * y.y + ap.y * y.x - ap.x * z.y - ap.y * z.x;
    }
    Z[e] = double2{sr, si};
  }
}

inline int grid_for(int64_t count) {
  int64_t g = (count + 255) / 256;
  return (int)std::min<int64_t>(std::max<int64_t>(g, 1), 65536);
}

// C = op(A) B (MODE 1) or C -= op(A) B (MODE 0), one product, general tiles
// ksp: K slices (slice s reads A + s kA, B + s kB and writes C + s kC)
template <int MODE>
void tri_gemm(hipStream_t st, int M, int N, int K, const double2* A, int64_t lda, bool conjA, const double2* B,
              int64_t ldb, double2* C, int64_t ldc, KSplit ksp = {1, 0, 0, 0}) {
  if (M <= 0 || N <= 0 || K <= 0) return;
  GemmOperand<double> a;
  a.p = A;
  a.stride = 0;
  a.ld = lda;
  a.conj = conjA ? 1 : 0;
  const unsigned gy = (unsigned)ksp.ks;
  if (N <= 16)
    hipLaunchKernelGGL((k_gemm<double, MODE, 64, 16, 4, 1>), dim3((unsigned)((M + 63) / 64), gy), dim3(256), 0, st, M,
                       N, K, a, a, 1, B, (int64_t)0, ldb, C, (int64_t)0, ldc, ksp);
  else
    hipLaunchKernelGGL((k_gemm<double, MODE, 64, 64, 2, 2>), dim3((unsigned)(((M + 63) / 64) * ((N + 63) / 64)), gy),
                       dim3(256), 0, st, M, N, K, a, a, 1, B, (int64_t)0, ldb, C, (int64_t)0, ldc, ksp);
}

}  // namespace

struct expm_pfd_tri_s {
  bool pooled = false;  // memory from the stream-ordered pool
  int64_t n = 0, npad = 0, m_max = 0;
  int degree = 0, P = 0, upper = 0, shift_t = 0;
  double shift = 0.0;
  bool factored = false;
  double2* Aw = nullptr;    // npad x npad: the Hermitian matrix being reduced, then the reflectors
  double2* Q = nullptr;     // npad x npad: Q of A = Q T Q^H
  double* d = nullptr;      // diagonal of T (n)
  double* e = nullptr;      // subdiagonal of T (n)
  double2* tau = nullptr;   // reflector scalars (n)
  double2* vbuf = nullptr;  // 2 x n: current and next reflector
  double2* y = nullptr;     // 2 x n: the products of two consecutive steps
  double2* part = nullptr;  // partial sums of the reduction's products
  double2* yv = nullptr;    // 2: their sums conj(y)^T v
  unsigned* done = nullptr;
  double2* Vp = nullptr;    // n x TRI_NB reflector panel
  double2* Tf = nullptr;    // TRI_NB x TRI_NB
  double2* Z1 = nullptr;    // TRI_NB x n
  double2* Z2 = nullptr;    // TRI_NB x n
  double2* Zp = nullptr;    // TRI_KS x TRI_NB x n: K-slice partial products
  double2* theta = nullptr;  // P
  double2* a = nullptr;      // P
  std::vector<double2> h_theta, h_a;
  double2* B = nullptr;     // n x m_max (row-major): Q^H V, then Z
  double2* Xr = nullptr;    // n x m_max (row-major): Q Z
  double2* Ysol = nullptr;  // n x (P 2 m_max)
  double2* Kp = nullptr;    // TRI_KS x n x m_max: K-slice partials of the products with Q
  double2* U = nullptr;     // n x (P 2 m_max): eliminated right-hand sides
  double2* F = nullptr;     // P x 2 x n x 3: the poles' tridiagonal factors
  ProblemDesc* desc = nullptr;
  double2* spk = nullptr;   // from order SPIKE_MIN_N: the spike solver's workspace
};

namespace {

void tri_free(expm_pfd_tri_t p, hipStream_t stream = nullptr) {
  if (!p) return;
  void* ptrs[] = {p->Aw, p->Q, p->d, p->e, p->tau, p->vbuf, p->y, p->part, p->yv, p->done, p->Vp, p->Tf,
                  p->Z1, p->Z2, p->Zp, p->theta, p->a, p->B, p->Xr, p->Ysol, p->Kp, p->U, p->F, p->desc, p->spk};
  for (void* q : ptrs)
    if (q) (void)(p->pooled ? hipFreeAsync(q, stream) : hipFree(q));
  delete p;
}

// byte counts of the plan's arrays, in allocation order
std::vector<size_t> tri_sizes(int64_t n, int degree, int64_t m_max) {
  const int64_t np = round_up(n, 64), P = degree / 2, nt = P * 2 * m_max;
  const int64_t nwg = (n + ROWS_PER_WG - 1) / ROWS_PER_WG;
  return {(size_t)np * np * 16, (size_t)(np + TRI_PAD) * np * 16, (size_t)n * 8, (size_t)n * 8, (size_t)n * 16,
          (size_t)2 * n * 16, (size_t)2 * n * 16, (size_t)nwg * 16, 32, 16, (size_t)(n + TRI_PAD) * TRI_NB * 16,
          (size_t)TRI_NB * TRI_NB * 16, (size_t)TRI_NB * n * 16, (size_t)TRI_NB * n * 16,
          (size_t)TRI_KS * TRI_NB * n * 16, (size_t)P * 16, (size_t)P * 16, (size_t)np * m_max * 16,
          (size_t)np * m_max * 16, (size_t)n * nt * 16, (size_t)TRI_KS * n * m_max * 16, (size_t)n * nt * 16,
          (size_t)n * P * 2 * 3 * 16, sizeof(ProblemDesc),
          n >= SPIKE_MIN_N ? spike_bytes(spike_plan(n, (int)P, (int)(2 * m_max)), (int)P) : 0};
}

}  // namespace

size_t expm::tri_bytes(int64_t n, int degree, int64_t m_max) {
  size_t b = 0;
  for (size_t x : tri_sizes(n, degree, m_max)) b += std::max<size_t>(x, 16);
  return b;
}

void expm::tri_release(expm_pfd_tri_t tri, hipStream_t stream) { tri_free(tri, stream); }

extern "C" int expm_pfd_tridiag_plan(expm_pfd_tri_t* out, int64_t n, int degree, int64_t m_max,
                                     const expm_pfd_opts* opts) {
  if (!out) return EXPM_PFD_ERR_NULL;
  *out = nullptr;
  if (int e = check_degree(degree)) return e;
  if (n < 1 || n > EXPM_PFD_MAX_N || m_max < 1 || m_max > 64 || m_max > n) return EXPM_PFD_ERR_DIM;
  if (int e = check_opts(opts)) return e;
  return tri_create(out, n, degree, m_max, opts, nullptr);
}

int expm::tri_create(expm_pfd_tri_t* out, int64_t n, int degree, int64_t m_max, const expm_pfd_opts* opts,
                     hipStream_t pool) {
  auto* p = new expm_pfd_tri_s();
  p->pooled = pool != nullptr;
  p->n = n;
  p->npad = round_up(n, 64);
  p->m_max = m_max;
  p->degree = degree;
  p->P = degree / 2;
  p->upper = opts ? opts->uplo : 0;
  p->shift = opts ? opts->shift : 0.0;
  p->shift_t = opts && opts->shift_scale_t ? 1 : 0;
  p->h_theta.resize(p->P);
  p->h_a.resize(p->P);
  if (int rc = expm_pfd_constants(degree, (double*)p->h_theta.data(), (double*)p->h_a.data())) {
    delete p;
    return rc;
  }
  const int64_t np = p->npad;
  bool ok = true;
  const std::vector<size_t> sz = tri_sizes(n, degree, m_max);
  size_t k = 0;
  auto dm = [&](auto** q) {
    const size_t bytes = std::max<size_t>(sz[k++], 16);
    ok = ok && (pool ? hipMallocAsync((void**)q, bytes, pool) : hipMalloc((void**)q, bytes)) == hipSuccess;
  };
  // (order and sizes: tri_sizes)
  dm(&p->Aw);
  dm(&p->Q);
  dm(&p->d);
  dm(&p->e);
  dm(&p->tau);
  dm(&p->vbuf);
  dm(&p->y);
  dm(&p->part);
  dm(&p->yv);
  dm(&p->done);
  dm(&p->Vp);
  dm(&p->Tf);
  dm(&p->Z1);
  dm(&p->Z2);
  dm(&p->Zp);
  dm(&p->theta);
  dm(&p->a);
  // B and Xr have npad rows, zero past n: the K slices of the products with Q
  // run over all npad rows (Q is zero there too)
  dm(&p->B);
  dm(&p->Xr);
  dm(&p->Ysol);
  dm(&p->Kp);
  dm(&p->U);
  dm(&p->F);  // one copy per workgroup of a pole (at most 2: 2 m_max <= 128)
  dm(&p->desc);
  dm(&p->spk);
  // the constants' host copies live in the plan, so the copies may complete later
  if (ok) ok = hipMemcpyAsync(p->theta, p->h_theta.data(), p->P * 16, hipMemcpyHostToDevice, pool) == hipSuccess;
  if (ok) ok = hipMemcpyAsync(p->a, p->h_a.data(), p->P * 16, hipMemcpyHostToDevice, pool) == hipSuccess;
  if (ok) ok = hipMemsetAsync(p->done, 0, 16, pool) == hipSuccess;
  if (ok && n >= SPIKE_MIN_N)  // the spike solver's zero poles
    ok = hipMemsetAsync(p->spk, 0, (size_t)p->P * 16, pool) == hipSuccess;
  if (ok) ok = hipMemsetAsync(p->B, 0, (size_t)np * m_max * 16, pool) == hipSuccess;
  if (ok) ok = hipMemsetAsync(p->Xr, 0, (size_t)np * m_max * 16, pool) == hipSuccess;
  if (ok && !pool) ok = hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    const bool oom = hipGetLastError() == hipErrorOutOfMemory;
    tri_free(p, pool);
    return oom ? EXPM_PFD_ERR_OOM : EXPM_PFD_ERR_HIP;
  }
  *out = p;
  return 0;
}

extern "C" int expm_pfd_tridiag_factor(expm_pfd_tri_t p, const void* A, int64_t lda, void* stream) {
  if (!p || !A) return EXPM_PFD_ERR_NULL;
  if (lda < p->n) return EXPM_PFD_ERR_LD;
  hipStream_t st = (hipStream_t)stream;
  const int n = (int)p->n;
  const int64_t ld = p->npad;
  (void)hipGetLastError();
  // the full Hermitian A (row-major) from the triangle read, by the shifted-matrix
  // formation kernel with no poles and t = 1
  {
    ProblemDesc one{};
    one.A = (const double2*)A;
    one.lda = lda;
    one.n = n;
    one.m = 1;
    one.t = 1.0;
    one.upper = p->upper;
    one.ec = 1.0;
    dim3 g((unsigned)(p->npad / 32), (unsigned)(p->npad / 32), 1), b(32, 8);
    hipLaunchKernelGGL((k_form<double>), g, b, 0, st, nullptr, one, (int)p->npad, p->theta, 0, (double2*)nullptr,
                       (int64_t)0, ld, p->Aw, ld);
  }
  if (n == 1) {
    hipLaunchKernelGGL(k_tri_eye, dim3(grid_for((ld + TRI_PAD) * ld)), dim3(256), 0, st, p->Q, ld, (int)ld + TRI_PAD,
                       n);
    hipLaunchKernelGGL(k_tri_order1, dim3(1), dim3(1), 0, st, p->Aw, p->d);
  } else {
    // step 0's product, then one fused launch per step (its update and the next
    // step's reflector and product), then the last step's update
    hipLaunchKernelGGL(k_tri_house0, dim3(1), dim3(64), 0, st, p->Aw, ld, n, p->vbuf, p->tau, p->e, p->d);
    {
      const unsigned g = (unsigned)((n - 1 + ROWS_PER_WG - 1) / ROWS_PER_WG);
      hipLaunchKernelGGL(k_tri_gemv, dim3(g), dim3(256), 0, st, p->Aw, ld, n, 0, p->vbuf, p->y, p->part, p->yv,
                         p->done);
    }
    for (int j = 0; j + 2 < n; ++j) {
      const int L = n - j - 1;
      const unsigned g = (unsigned)((L - 1 + FUSED_ROWS - 1) / FUSED_ROWS);
      const int b = j & 1, bn = (j + 1) & 1;
      hipLaunchKernelGGL(k_tri_step, dim3(g), dim3(FUSED_NT), (size_t)L * sizeof(double2), st, p->Aw, ld, n, j,
                         p->vbuf + b * n, p->vbuf + bn * n, p->y + b * n, p->y + bn * n, p->yv + b, p->yv + bn,
                         p->tau, p->e, p->d, p->part, p->done);
    }
    {
      const int j = n - 2, b = j & 1;
      hipLaunchKernelGGL(k_tri_update, dim3(1), dim3(256), 0, st, p->Aw, ld, n, j, p->vbuf + b * n,
                         p->vbuf + ((j + 1) & 1) * n, p->y + b * n, p->yv + b, p->tau, p->e, p->d);
    }
    // Q = H_0 H_1 ... H_{n-2}, accumulated backwards in blocks of TRI_NB reflectors
    hipLaunchKernelGGL(k_tri_eye, dim3(grid_for((ld + TRI_PAD) * ld)), dim3(256), 0, st, p->Q, ld, (int)ld + TRI_PAD,
                       n);
    const int nref = n - 1;
    for (int j0 = ((nref - 1) / TRI_NB) * TRI_NB; j0 >= 0; j0 -= TRI_NB) {
      const int nb = std::min(TRI_NB, nref - j0);
      const int L = n - j0 - 1;
      // the reductions over the L rows (V^H V, V^H Qs) in ks K slices of Ks rows;
      // the panel and Q carry zero rows past L, so the padded slices add zeros
      const int ks = std::max(1, std::min(TRI_KS, (L + 127) / 128));
      const int Ks = (int)round_up((L + ks - 1) / ks, 16);
      const int Lpad = ks * Ks;
      hipLaunchKernelGGL(k_tri_vpanel, dim3(grid_for((int64_t)Lpad * nb)), dim3(256), 0, st, p->Aw, ld, n, j0, nb,
                         Lpad, p->Vp);
      double2* Qs = p->Q + (int64_t)(j0 + 1) * ld + (j0 + 1);
      // S = V^H V, then T
      tri_gemm<1>(st, nb, nb, Ks, p->Vp, nb, true, p->Vp, nb, p->Zp, nb,
                  KSplit{ks, (int64_t)Ks * nb, (int64_t)Ks * nb, (int64_t)nb * nb});
      hipLaunchKernelGGL(k_tri_sum_slices, dim3(grid_for((int64_t)nb * nb)), dim3(256), 0, st, p->Zp, ks,
                         (int64_t)nb * nb, (int64_t)nb * nb, p->Z2);
      hipLaunchKernelGGL(k_tri_tfactor, dim3(1), dim3(64), 0, st, p->Z2, nb, p->tau + j0, p->Tf);
      // Z1 = V^H Qs, Z2 = T Z1, Qs -= V Z2
      tri_gemm<1>(st, nb, L, Ks, p->Vp, nb, true, Qs, ld, p->Zp, L,
                  KSplit{ks, (int64_t)Ks * nb, (int64_t)Ks * ld, (int64_t)nb * L});
      hipLaunchKernelGGL(k_tri_sum_slices, dim3(grid_for((int64_t)nb * L)), dim3(256), 0, st, p->Zp, ks,
                         (int64_t)nb * L, (int64_t)nb * L, p->Z1);
      tri_gemm<1>(st, nb, L, nb, p->Tf, nb, false, p->Z1, L, p->Z2, L);
      tri_gemm<0>(st, L, L, nb, p->Vp, nb, false, p->Z2, L, Qs, ld);
    }
  }
  if (hipGetLastError() != hipSuccess) return EXPM_PFD_ERR_HIP;
  p->factored = true;
  return 0;
}

extern "C" int expm_pfd_tridiag_apply(expm_pfd_tri_t p, double t, const void* V, int64_t ldv, int64_t m, void* X,
                                      int64_t ldx, void* stream) {
  if (!p || !V || !X) return EXPM_PFD_ERR_NULL;
  if (!p->factored) return EXPM_PFD_ERR_ARG;
  if (!std::isfinite(t)) return EXPM_PFD_ERR_ARG;
  if (m < 1 || m > p->m_max) return EXPM_PFD_ERR_DIM;
  if (ldv < p->n || ldx < p->n) return EXPM_PFD_ERR_LD;
  ProblemDesc sh{};
  if (problem_shift(p->shift, p->shift_t, t, sh)) return EXPM_PFD_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int n = (int)p->n, mm = (int)m;
  const int64_t ld = p->npad;
  (void)hipGetLastError();
  // B = Q^H V (V staged row-major in Xr)
  hipLaunchKernelGGL(k_tri_layout, dim3(grid_for((int64_t)n * mm)), dim3(256), 0, st, (const double2*)V, ldv, p->Xr,
                     (int64_t)mm, n, mm, 0);
  // the products with Q (n x npad x m) in K slices: ks | npad/16, partials summed in order
  int ks = 1;
  while (ks < TRI_KS && ld % (32 * ks) == 0 && ld / (2 * ks) >= 128) ks *= 2;
  const int Ks = (int)(ld / ks);
  tri_gemm<1>(st, n, mm, Ks, p->Q, ld, true, p->Xr, mm, p->Kp, mm,
              KSplit{ks, (int64_t)Ks * ld, (int64_t)Ks * mm, (int64_t)n * mm});
  hipLaunchKernelGGL(k_tri_sum_slices, dim3(grid_for((int64_t)n * mm)), dim3(256), 0, st, p->Kp, ks,
                     (int64_t)n * mm, (int64_t)n * mm, p->B);
  const int nt = p->P * 2 * mm;
  if (n >= SPIKE_MIN_N) {
    SpikeSrc src{};
    src.kind = 1;
    src.d = p->d;
    src.e = p->e;
    src.t = t;
    src.c = sh.c;
    src.V = p->B;
    src.mv = mm;
    src.ncol = 2 * mm;
    src.n = n;
    const SpikePlan q = spike_plan(n, p->P, 2 * mm);
    spike_solve(src, p->theta, p->P, q, spike_carve(p->spk, q, p->P), SpikeOutInterleaved{p->Ysol, nt, 2 * mm}, st);
  } else {
    hipLaunchKernelGGL(k_tri_solve, dim3((unsigned)p->P, (unsigned)((2 * mm + 63) / 64)), dim3(64), 0, st, p->d,
                       p->e, n, t, p->theta, p->P, sh.c, p->B, mm, p->F, p->U, p->Ysol);
  }
  hipLaunchKernelGGL(k_tri_accum, dim3(grid_for((int64_t)n * mm)), dim3(256), 0, st, p->Ysol, n, mm, p->P, p->a,
                     sh.ec, p->B);
  tri_gemm<1>(st, n, mm, Ks, p->Q, ld, false, p->B, mm, p->Kp, mm,
              KSplit{ks, (int64_t)Ks, (int64_t)Ks * mm, (int64_t)n * mm});
  hipLaunchKernelGGL(k_tri_sum_slices, dim3(grid_for((int64_t)n * mm)), dim3(256), 0, st, p->Kp, ks,
                     (int64_t)n * mm, (int64_t)n * mm, p->Xr);
  hipLaunchKernelGGL(k_tri_layout, dim3(grid_for((int64_t)n * mm)), dim3(256), 0, st, p->Xr, (int64_t)mm,
                     (double2*)X, ldx, n, mm, 1);
  return hipGetLastError() == hipSuccess ? 0 : EXPM_PFD_ERR_HIP;
}

extern "C" int expm_pfd_tridiag_diagonals(expm_pfd_tri_t p, double* d, double* e) {
  if (!p || !d || !e) return EXPM_PFD_ERR_NULL;
  if (!p->factored) return EXPM_PFD_ERR_ARG;
  if (hipDeviceSynchronize() != hipSuccess) return EXPM_PFD_ERR_HIP;
  if (hipMemcpy(d, p->d, (size_t)p->n * 8, hipMemcpyDeviceToHost) != hipSuccess) return EXPM_PFD_ERR_HIP;
  if (p->n > 1 && hipMemcpy(e, p->e, (size_t)(p->n - 1) * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return EXPM_PFD_ERR_HIP;
  return 0;
}

extern "C" int expm_pfd_tridiag_destroy(expm_pfd_tri_t p) {
  if (!p) return EXPM_PFD_ERR_NULL;
  (void)hipDeviceSynchronize();
  tri_free(p);
  return 0;
}

// Partitioned solution of the per-pole tridiagonal systems (M + theta_k I) x = f of
// the tridiagonal and banded (kd = 1) routes (eq. equ:expAx with a tridiagonal
// shifted matrix).  Eliminating a tridiagonal system row by row is a chain of n
// dependent steps; here the rows are cut into P segments that are eliminated side by
// side (one lane per segment and column), then joined through a small system on the
// segment boundaries (the spike method):
//   M_i y_i = f_i,  M_i v_i = M(hi-1, hi) e_last,  M_i w_i = M(lo, lo-1) e_first,
//   x_i = y_i - v_i x(hi) - w_i x(lo-1),
// where M_i is the diagonal block of segment i = [lo, hi).  Writing a_i = x(lo_i) and
// b_i = x(hi_i - 1), the rows lo and hi-1 of the last line give 2P equations in the
// unknowns (a_0, b_0, a_1, b_1, ...), a band matrix with two sub- and two
// superdiagonals, solved by the one-wave band kernel; then every row is corrected in
// parallel.  Each segment is eliminated with partial pivoting inside it: its block is
// tT_i + theta I (or tA_i - cI + theta I) with T_i real symmetric (A_i Hermitian), so
// it is nonsingular for Im theta != 0, and the boundary system is nonsingular with M.
// Included by one translation unit each; everything is internal.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "band_chain.h"

namespace {

// The tridiagonal matrix and right-hand sides of one apply.
struct SpikeSrc {
  int kind;  // 0: complex rows R[j*3 + c] = M(j, j-1+c) of tA - cI; 1: real symmetric (d, e) of T, times t, minus c
  const double2* R;
  const double* d;
  const double* e;
  double t, c;
  const double2* V;  // kind 0: V[j*mv + r]; kind 1: B[j*mv + (r mod mv)], conjugated for r >= mv
  int mv;
  int ncol;  // right-hand sides per pole (kind 0: m; kind 1: 2m, the conjugate pole's through conj(B))
  int n;
};

__device__ __forceinline__ double2 sp_diag(const SpikeSrc& s, double2 th, int j) {
  double2 v;
  if (s.kind == 0) {
    v = s.R[(int64_t)j * 3 + 1];
  } else {
    v.x = s.t * s.d[j] - s.c;
    v.y = 0.0;
  }
  v.x += th.x;
  v.y += th.y;
  return v;
}
__device__ __forceinline__ double2 sp_sub(const SpikeSrc& s, int j) {  // M(j+1, j)
  if (s.kind == 0) return s.R[(int64_t)(j + 1) * 3];
  return double2{s.t * s.e[j], 0.0};
}
__device__ __forceinline__ double2 sp_sup(const SpikeSrc& s, int j) {  // M(j, j+1)
  if (s.kind == 0) return s.R[(int64_t)j * 3 + 2];
  return double2{s.t * s.e[j], 0.0};
}
__device__ __forceinline__ double2 sp_rhs(const SpikeSrc& s, int j, int r) {
  if (s.kind == 0) return s.V[(int64_t)j * s.mv + r];
  double2 b = s.V[(int64_t)j * s.mv + (r % s.mv)];
  if (r >= s.mv) b.y = -b.y;
  return b;
}
__device__ __forceinline__ int seg_lo(int i, int n, int P) { return (int)((int64_t)i * n / P); }

// One lane per (pole, segment, column): the segment's elimination with partial
// pivoting applied to the column, then its back substitution.  Columns 0..ncol-1
// are the right-hand sides, ncol the right spike v, ncol+1 the left spike w.
// Y (ld = ncol + 2) receives the forward-eliminated column and then the solution
// in place; F the rows of U (1/pivot, u1, u2), one copy per column.
__global__ __launch_bounds__(64) void k_spike_seg(SpikeSrc s, const double2* __restrict__ pole, int P,
                                                  double2* __restrict__ Yb, double2* __restrict__ Fb,
                                                  int64_t ystride, int64_t fstride) {
  const int k = blockIdx.y;
  const int ld = s.ncol + 2;
  const int idx = blockIdx.x * 64 + threadIdx.x;
  if (idx >= P * ld) return;  // (no wave-wide operations below)
  const int i = idx / ld, col = idx % ld;
  const int n = s.n, lo = seg_lo(i, n, P), hi = seg_lo(i + 1, n, P);
  const double2 th = pole[k];
  double2* Y = Yb + k * ystride + col;
  double2* F = Fb + k * fstride + (int64_t)col * 3;
  const double2 zero = czero<double2>();
  auto rhs = [&](int j) {
    if (col < s.ncol) return sp_rhs(s, j, col);
    if (col == s.ncol) return (j == hi - 1 && hi < n) ? sp_sup(s, j) : zero;  // coupling M(hi-1, hi)
    return (j == lo && lo > 0) ? sp_sub(s, lo - 1) : zero;                    // coupling M(lo, lo-1)
  };
  // the carry row (after the previous eliminations) has entries cp (column j) and
  // cq (column j+1); the next row of the segment, (off, dn, offn) at j, j+1, j+2
  double2 cp = sp_diag(s, th, lo), cq = lo + 1 < hi ? sp_sup(s, lo) : zero, cb = rhs(lo);
  // inputs of step j loaded one step ahead
  double2 off_n = zero, dn_n = zero, offn_n = zero, bn_n = zero;
  if (lo + 1 < hi) {
    off_n = sp_sub(s, lo);
    dn_n = sp_diag(s, th, lo + 1);
    offn_n = lo + 2 < hi ? sp_sup(s, lo + 1) : zero;
    bn_n = rhs(lo + 1);
  }
  for (int j = lo; j + 1 < hi; ++j) {
    const double2 off = off_n, dn = dn_n, offn = offn_n, bn = bn_n;
    if (j + 2 < hi) {
      off_n = sp_sub(s, j + 1);
      dn_n = sp_diag(s, th, j + 2);
      offn_n = j + 3 < hi ? sp_sup(s, j + 2) : zero;
      bn_n = rhs(j + 2);
    }
    const bool sw = pivot_mag(off) > pivot_mag(cp);
    const double2 piv = sw ? off : cp, u1 = sw ? dn : cq, u2 = sw ? offn : zero, ub = sw ? bn : cb;
    const double2 o0 = sw ? cp : off, o1 = sw ? cq : dn, o2 = sw ? zero : offn, ob = sw ? cb : bn;
    const double2 rp = crecip_fast(piv);
    const double2 l = cmul(o0, rp);
    double2* Fj = F + (int64_t)j * ld * 3;
    Fj[0] = rp;
    Fj[1] = u1;
    Fj[2] = u2;
    Y[(int64_t)j * ld] = ub;
    cp = cfms(o1, l, u1);
    cq = cfms(o2, l, u2);
    cb = cfms(ob, l, ub);
  }
  double2 x1 = cmul(cb, crecip_fast(cp)), x2 = zero;
  Y[(int64_t)(hi - 1) * ld] = x1;
  for (int j = hi - 2; j >= lo; --j) {
    const double2* Fj = F + (int64_t)j * ld * 3;
    double2 v = cfms(Y[(int64_t)j * ld], Fj[1], x1);
    v = cfms(v, Fj[2], x2);
    const double2 x = cmul(v, Fj[0]);
    Y[(int64_t)j * ld] = x;
    x2 = x1;
    x1 = x;
  }
}

// The boundary system of each pole: band rows (kd = 2, row-major, 5 per row) and
// right-hand sides (2P x ncol, row-major) from the segments' first and last rows.
// grid (ceil(P*ncol / 256), poles), block 256
__global__ __launch_bounds__(256) void k_spike_reduce(int n, int ncol, int P, const double2* __restrict__ Yb,
                                                      int64_t ystride, double2* __restrict__ Z5b,
                                                      double2* __restrict__ Zvb, int64_t zstride5,
                                                      int64_t zstridev) {
  const int k = blockIdx.y;
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= P * ncol) return;
  const int i = idx / ncol, r = idx % ncol, ld = ncol + 2;
  const int lo = seg_lo(i, n, P), last = seg_lo(i + 1, n, P) - 1;
  const double2* Y = Yb + k * ystride;
  double2* Zv = Zvb + k * zstridev;
  Zv[(int64_t)(2 * i) * ncol + r] = Y[(int64_t)lo * ld + r];
  Zv[(int64_t)(2 * i + 1) * ncol + r] = Y[(int64_t)last * ld + r];
  if (r == 0) {
    double2* Z5 = Z5b + k * zstride5 + (int64_t)(2 * i) * 5;
    const double2 zero = czero<double2>(), one = double2{1.0, 0.0};
    // row a_i: columns 2i-2 .. 2i+2: (0, w_i(lo), 1, 0, v_i(lo))
    Z5[0] = zero;
    Z5[1] = Y[(int64_t)lo * ld + ncol + 1];
    Z5[2] = one;
    Z5[3] = zero;
    Z5[4] = Y[(int64_t)lo * ld + ncol];
    // row b_i: columns 2i-1 .. 2i+3: (w_i(hi-1), 0, 1, v_i(hi-1), 0)
    Z5[5] = Y[(int64_t)last * ld + ncol + 1];
    Z5[6] = zero;
    Z5[7] = one;
    Z5[8] = Y[(int64_t)last * ld + ncol];
    Z5[9] = zero;
  }
}

// x_j = y_j - v_j a_{i+1} - w_j b_{i-1} for row j of segment i, written through
// `out(k, j, r, x)`.  grid (ceil(n*ncol / 256), poles), block 256
template <typename Out>
__global__ __launch_bounds__(256) void k_spike_fix(int n, int ncol, int P, const double2* __restrict__ Yb,
                                                   int64_t ystride, const double2* __restrict__ Zsb, int64_t zstride,
                                                   Out out) {
  const int k = blockIdx.y;
  const int64_t idx = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (idx >= (int64_t)n * ncol) return;
  const int j = (int)(idx / ncol), r = (int)(idx % ncol), ld = ncol + 2;
  const int i = (int)(((int64_t)(j + 1) * P - 1) / n);  // the segment of row j
  const double2* Y = Yb + k * ystride + (int64_t)j * ld;
  double2 x = Y[r];
  if (P > 1) {
    const double2* Zs = Zsb + k * zstride;
    if (i + 1 < P) x = cfms(x, Y[ncol], Zs[(int64_t)(2 * i + 2) * ncol + r]);
    if (i > 0) x = cfms(x, Y[ncol + 1], Zs[(int64_t)(2 * i - 1) * ncol + r]);
  }
  out(k, j, r, x);
}

// Workspace of the spike solver for S poles, order n, at most ncol columns.
struct SpikePlan {
  int P = 1;
  int64_t ystride = 0, fstride = 0, z5stride = 0, zvstride = 0, ustride = 0;
  size_t y_elems = 0, f_elems = 0, z5_elems = 0, zv_elems = 0, u_elems = 0;
};
inline SpikePlan spike_plan(int64_t n, int S, int ncol) {
  SpikePlan q;
  // segments of about max(64, sqrt(2n)) rows, at least two rows each
  const int64_t b = std::max<int64_t>(64, (int64_t)std::sqrt(2.0 * (double)n));
  q.P = (int)std::max<int64_t>(1, std::min<int64_t>(n / b, n / 2));
  const int64_t ld = ncol + 2, nr = 2 * (int64_t)q.P;
  q.ystride = n * ld;
  q.fstride = n * ld * 3;
  q.z5stride = nr * 5;
  q.zvstride = nr * ncol;
  const int64_t chunks = (ncol + NB_MC - 1) / NB_MC;
  q.ustride = nr * 5;
  q.y_elems = (size_t)S * q.ystride;
  q.f_elems = (size_t)S * q.fstride;
  q.z5_elems = (size_t)S * q.z5stride;
  q.zv_elems = (size_t)S * q.zvstride;  // (right-hand sides; the solution has the same size)
  q.u_elems = (size_t)S * chunks * q.ustride;
  return q;
}
inline size_t spike_bytes(const SpikePlan& q, int S) {
  return (q.y_elems + q.f_elems + q.z5_elems + 2 * q.zv_elems + q.u_elems + (size_t)S) * sizeof(double2);
}

// Buffers of one spike workspace (device pointers, sizes from spike_plan).
struct SpikeBufs {
  double2 *Y = nullptr, *F = nullptr, *Z5 = nullptr, *Zv = nullptr, *Zs = nullptr, *U = nullptr, *zero = nullptr;
};
// The buffers carved from one allocation of spike_bytes(plan for the largest ncol):
// S zero poles first (cleared once, the same place for every ncol), then the rest.
inline SpikeBufs spike_carve(double2* base, const SpikePlan& q, int S) {
  SpikeBufs b;
  double2* p = base;
  b.zero = p;
  p += S;
  b.Y = p;
  p += q.y_elems;
  b.F = p;
  p += q.f_elems;
  b.Z5 = p;
  p += q.z5_elems;
  b.Zv = p;
  p += q.zv_elems;
  b.Zs = p;
  p += q.zv_elems;
  b.U = p;
  return b;
}

// Output of a solution entry: pole k's n x m block, row-major (banded route)
struct SpikeOutRows {
  double2* Y;
  int64_t ystride;
  int m;
  __device__ __forceinline__ void operator()(int k, int j, int r, double2 x) const {
    Y[k * ystride + (int64_t)j * m + r] = x;
  }
};
// ... or row j of one n x (poles x ncol) array (tridiagonal route)
struct SpikeOutInterleaved {
  double2* Y;
  int64_t nt;
  int ncol;
  __device__ __forceinline__ void operator()(int k, int j, int r, double2 x) const {
    Y[(int64_t)j * nt + (int64_t)k * ncol + r] = x;
  }
};

// the spike solver is used from this order on (shorter chains are eliminated whole)
constexpr int64_t SPIKE_MIN_N = 128;

// All launches of one spike solve on stream st.
template <typename Out>
inline void spike_solve(const SpikeSrc& s, const double2* pole, int S, const SpikePlan& q, const SpikeBufs& b,
                        Out out, hipStream_t st) {
  const int ld = s.ncol + 2;
  hipLaunchKernelGGL(k_spike_seg, dim3((unsigned)((q.P * ld + 63) / 64), (unsigned)S), dim3(64), 0, st, s, pole, q.P,
                     b.Y, b.F, q.ystride, q.fstride);
  if (q.P > 1) {
    hipLaunchKernelGGL(k_spike_reduce, dim3((unsigned)((q.P * s.ncol + 255) / 256), (unsigned)S), dim3(256), 0, st,
                       s.n, s.ncol, q.P, b.Y, q.ystride, b.Z5, b.Zv, q.z5stride, q.zvstride);
    const dim3 g((unsigned)S, (unsigned)((s.ncol + NB_MC - 1) / NB_MC));
    hipLaunchKernelGGL(k_band_narrow<2>, g, dim3(64), 0, st, 2 * q.P, s.ncol, b.Z5, b.Zv, b.zero, b.U, b.Zs,
                       q.ustride, q.zvstride, q.z5stride, q.zvstride);
  }
  hipLaunchKernelGGL(k_spike_fix<Out>, dim3((unsigned)(((int64_t)s.n * s.ncol + 255) / 256), (unsigned)S), dim3(256),
                     0, st, s.n, s.ncol, q.P, b.Y, q.ystride, b.Zs, q.zvstride, out);
}

}  // namespace

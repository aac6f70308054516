// Kernels of the exp(tA)V hot path on gfx950.
//
// Storage used by every kernel below: the shifted matrices M_k = tA + theta_k I,
// their LU factors and the right-hand-side blocks are ROW-major complex arrays
// (element (i, j) at base[i*ld + j]) of padded order npad (a multiple of 64).
// The padding is the identity (matrix) or zero (right-hand sides), so it never
// interacts with the n x n problem.  Row-major storage makes a row interchange a
// contiguous copy and keeps every pivot-row access coalesced.
#pragma once

#include "device_common.h"

namespace expm {

// ---------------------------------------------------------------------------
// K1: form the shifted matrices  W_p = t*A + theta_p I  (paper Sec. 3,
// eqs. equ:ExpoMatRat and equ:expAx: one shifted matrix per pole; with the
// conjugate pairs of Remark rem:two_time_real_part one per pair suffices).
// A is column-major, lower triangle read; the Hermitian operand is built here
// so that W_p for conj(theta_p) would be exactly W_p^H.  The shift is added in
// FP64 before any rounding to the working type.  Optionally also writes
// Ah = t*A (full Hermitian, FP64, row-major) for the refinement residuals.
// grid (npad/32, npad/32), block (32, 8)
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_form(const double2* __restrict__ A, int64_t lda, int n, int npad,
                                              double t, const double2* __restrict__ theta, int P,
                                              cx<R>* __restrict__ W, int64_t wstride, int64_t ldw,
                                              double2* __restrict__ Ah, int64_t ldh) {
  __shared__ double2 tile[32][33];
  const int bi = blockIdx.y, bj = blockIdx.x;
  const int R0 = (bi > bj ? bi : bj) * 32, C0 = (bi < bj ? bi : bj) * 32;
  for (int cc = threadIdx.y; cc < 32; cc += 8) {
    const int r = R0 + threadIdx.x, c = C0 + cc;
    double2 v = czero<double2>();
    if (r < n && c < n) v = A[r + (int64_t)c * lda];
    tile[cc][threadIdx.x] = v;
  }
  __syncthreads();
  for (int ry = threadIdx.y; ry < 32; ry += 8) {
    const int r = bi * 32 + ry, c = bj * 32 + threadIdx.x;
    double2 v;
    if (r >= n || c >= n) {
      v = czero<double2>();
    } else if (r > c) {
      v = tile[c - C0][r - R0];
    } else if (r < c) {
      v = cconj(tile[r - C0][c - R0]);
    } else {
      v.x = tile[c - C0][r - R0].x;
      v.y = 0;
    }
    v.x *= t;
    v.y *= t;
    if (Ah) Ah[(int64_t)r * ldh + c] = v;
    for (int p = 0; p < P; ++p) {
      double2 w = v;
      if (r == c) {
        if (r < n) {
          w.x += theta[p].x;
          w.y += theta[p].y;
        } else {
          w.x = 1;
          w.y = 0;
        }
      }
      cx<R> o;
      o.x = (R)w.x;
      o.y = (R)w.y;
      W[p * wstride + (int64_t)r * ldw + c] = o;
    }
  }
}

// ---------------------------------------------------------------------------
// K2: panel factorization with partial pivoting (LAPACK getf2 order) of the
// IB columns [c0, c0+IB) over rows [c0, npad), for one shifted matrix per
// workgroup.  The panel lives in registers: thread t owns rows c0+t+1024s.
// Per column: pivot = argmax |Re|+|Im| (lowest row on ties) by wave reductions
// and one LDS exchange, pivot row broadcast through LDS, rank-1 update in
// registers (two barriers per column).
// Then, inside the enclosing outer panel [j0, j0+nbo): the IB interchanges are
// applied to the other outer-panel columns and the IB x (rest) block of U is
// solved with the unit lower IB x IB factor.  If this is the last inner step,
// the net row moves of the whole outer step are written for later use.
// grid (P), block 1024
// ---------------------------------------------------------------------------
template <typename R, int IB, int S>
__global__ __launch_bounds__(1024) void k_panel(cx<R>* __restrict__ Wb, int64_t wstride, int64_t ld, int npad, int j0,
                                                int c0, int nbo, int* __restrict__ ipivb, int64_t pstride,
                                                int* __restrict__ movesb, int64_t mstride, int step, int last) {
  using T = cx<R>;
  __shared__ R red_v[2][16];
  __shared__ int red_i[2][16];
  __shared__ T prow[2][IB];
  __shared__ T crow[2][IB];
  __shared__ T Lib[IB][IB + 1];
  __shared__ T mvbuf[2 * IB][NB_MAX];
  __shared__ int mv_dst[MOVE_CAP], mv_src[MOVE_CAP];
  __shared__ int mv_cnt;

  const int b = blockIdx.x;
  T* W = Wb + b * wstride;
  int* ipiv = ipivb + b * pstride;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;

  T a[S][IB];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int r = c0 + tid + 1024 * s;
#pragma unroll
    for (int c = 0; c < IB; ++c) a[s][c] = (r < npad) ? W[(int64_t)r * ld + c0 + c] : czero<T>();
  }

#pragma unroll
  for (int c = 0; c < IB; ++c) {
    const int gc = c0 + c, buf = c & 1;
    R bv = -1;
    int bi = 0x7fffffff;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int r = c0 + tid + 1024 * s;
      if (r >= gc && r < npad) {
        const R v = fabs(a[s][c].x) + fabs(a[s][c].y);
        if (v > bv) {
          bv = v;
          bi = r;
        }
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const R ov = __shfl_xor(bv, off);
      const int oi = __shfl_xor(bi, off);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      red_v[buf][wid] = bv;
      red_i[buf][wid] = bi;
    }
    __syncthreads();
    bv = red_v[buf][0];
    bi = red_i[buf][0];
#pragma unroll
    for (int w = 1; w < 16; ++w) {
      const R ov = red_v[buf][w];
      const int oi = red_i[buf][w];
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    const int p = bi;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int r = c0 + tid + 1024 * s;
      if (r == p) {
#pragma unroll
        for (int cc = 0; cc < IB; ++cc) prow[buf][cc] = a[s][cc];
      }
      if (r == gc && p != gc) {
#pragma unroll
        for (int cc = 0; cc < IB; ++cc) crow[buf][cc] = a[s][cc];
      }
    }
    __syncthreads();
    // the pivot row is read from LDS where needed (broadcast reads), not held in registers
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int r = c0 + tid + 1024 * s;
      if (r == gc) {
#pragma unroll
        for (int cc = 0; cc < IB; ++cc) a[s][cc] = prow[buf][cc];
      } else if (r == p) {
#pragma unroll
        for (int cc = 0; cc < IB; ++cc) a[s][cc] = crow[buf][cc];
      }
    }
    const T inv = crecip(prow[buf][c]);
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int r = c0 + tid + 1024 * s;
      if (r > gc && r < npad) {
        const T l = cmul(a[s][c], inv);
        a[s][c] = l;
#pragma unroll
        for (int cc = c + 1; cc < IB; ++cc) a[s][cc] = cfms(a[s][cc], l, prow[buf][cc]);
      }
    }
    if (tid == 0) ipiv[gc] = p;
  }

#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int r = c0 + tid + 1024 * s;
    if (r < npad) {
#pragma unroll
      for (int c = 0; c < IB; ++c) W[(int64_t)r * ld + c0 + c] = a[s][c];
    }
  }
  __syncthreads();

  // ---- interchanges on the other columns of the outer panel, then U block --
  if (wid == 0) {
    const int cnt = composite_moves(ipiv + c0, IB, c0, mv_dst, mv_src);
    if (lane == 0) mv_cnt = cnt;
  }
  if (tid < IB * IB) {
    const int i = tid / IB, k = tid % IB;
    Lib[i][k] = W[(int64_t)(c0 + i) * ld + c0 + k];
  }
  __syncthreads();
  const int nleft = c0 - j0, nright = j0 + nbo - c0 - IB, nother = nleft + nright;
  const int cnt = mv_cnt;
  for (int e = tid; e < cnt * nother; e += 1024) {
    const int i = e / nother, cc = e % nother;
    const int col = cc < nleft ? j0 + cc : c0 + IB + (cc - nleft);
    mvbuf[i][cc] = W[(int64_t)mv_src[i] * ld + col];
  }
  __syncthreads();
  for (int e = tid; e < cnt * nother; e += 1024) {
    const int i = e / nother, cc = e % nother;
    const int col = cc < nleft ? j0 + cc : c0 + IB + (cc - nleft);
    W[(int64_t)mv_dst[i] * ld + col] = mvbuf[i][cc];
  }
  __syncthreads();
  if (tid < nright) {
    const int col = c0 + IB + tid;
    T x[IB];
#pragma unroll
    for (int i = 0; i < IB; ++i) x[i] = W[(int64_t)(c0 + i) * ld + col];
#pragma unroll
    for (int i = 1; i < IB; ++i)
#pragma unroll
      for (int k = 0; k < i; ++k) x[i] = cfms(x[i], Lib[i][k], x[k]);
#pragma unroll
    for (int i = 1; i < IB; ++i) W[(int64_t)(c0 + i) * ld + col] = x[i];
  }
  if (last && wid == 0) {
    int* mv = movesb + b * mstride + (int64_t)step * MOVE_STRIDE;
    const int cnt2 = composite_moves(ipiv + j0, nbo, j0, mv + 1, mv + 1 + MOVE_CAP);
    if (lane == 0) mv[0] = cnt2;
  }
}

// ---------------------------------------------------------------------------
// K5: C -= op(A) * B for complex matrices on the matrix cores, batched over
// blockIdx.y.  op(A) = A (row-major M x K, lda) or, with CONJA, the conjugate
// transpose of a row-major K x M array.  B row-major K x N, C row-major M x N.
// Complex products from real 16x16x4 products: the K dimension is interleaved
// (real index 2k = real part, 2k+1 = imaginary part), so with b = (Re B, Im B)
// per k, Re C uses a = (Re A, -Im A) and Im C uses a = (Im A, Re A): two real
// products per 16x16 complex block and pair of k, B operand shared.
// Tiles BM x BN per 256-thread workgroup, waves WGM x WGN, K staged through LDS
// in chunks of 16.
// ---------------------------------------------------------------------------
template <typename R, bool CONJA, int BM, int BN, int WGM, int WGN>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const cx<R>* __restrict__ A, int64_t sA,
                                              int64_t lda, const cx<R>* __restrict__ B, int64_t sB, int64_t ldb,
                                              cx<R>* __restrict__ C, int64_t sC, int64_t ldc) {
  using T = cx<R>;
  using MF = Mfma<R>;
  using V = typename MF::V;
  constexpr int KC = 16;
  constexpr int WM = BM / WGM, WN = BN / WGN, MI = WM / 16, NJ = WN / 16;
  static_assert(WGM * WGN == 4, "four waves");
  __shared__ T As[BM][KC + 1];
  __shared__ T Bs[KC][BN + 1];

  const int tiles_m = (M + BM - 1) / BM;
  const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
  const int bb = blockIdx.y;
  A += bb * sA;
  B += bb * sB;
  C += bb * sC;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm0 = (w / WGN) * WM, wn0 = (w % WGN) * WN;
  const int r16 = lane & 15, kq = lane >> 4;
  const int m0 = tm * BM, n0 = tn * BN;

  V accR[MI][NJ], accI[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      accR[i][j] = V{0, 0, 0, 0};
      accI[i][j] = V{0, 0, 0, 0};
    }

  for (int k0 = 0; k0 < K; k0 += KC) {
    if (!CONJA) {
      for (int e = tid; e < BM * KC; e += 256) {
        const int i = e / KC, k = e % KC;
        T v = czero<T>();
        if (m0 + i < M && k0 + k < K) v = A[(int64_t)(m0 + i) * lda + k0 + k];
        As[i][k] = v;
      }
    } else {
      for (int e = tid; e < BM * KC; e += 256) {
        const int i = e % BM, k = e / BM;
        T v = czero<T>();
        if (m0 + i < M && k0 + k < K) v = cconj(A[(int64_t)(k0 + k) * lda + m0 + i]);
        As[i][k] = v;
      }
    }
    for (int e = tid; e < KC * BN; e += 256) {
      const int j = e % BN, k = e / BN;
      T v = czero<T>();
      if (n0 + j < N && k0 + k < K) v = B[(int64_t)(k0 + k) * ldb + n0 + j];
      Bs[k][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k2 = 0; k2 < KC / 2; ++k2) {
      const int kc = 2 * k2 + (kq >> 1);
      const bool odd = kq & 1;
      R aR[MI], aI[MI], bR[NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        const T av = As[wm0 + i * 16 + r16][kc];
        aR[i] = odd ? -av.y : av.x;
        aI[i] = odd ? av.x : av.y;
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const T bv = Bs[kc][wn0 + j * 16 + r16];
        bR[j] = odd ? bv.y : bv.x;
      }
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          accR[i][j] = MF::run(aR[i], bR[j], accR[i][j]);
          accI[i][j] = MF::run(aI[i], bR[j], accI[i][j]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm0 + i * 16 + MF::row(kq, r);
        const int col = n0 + wn0 + j * 16 + r16;
        if (row < M && col < N) {
          T c = C[(int64_t)row * ldc + col];
          c.x -= accR[i][j][r];
          c.y -= accI[i][j][r];
          C[(int64_t)row * ldc + col] = c;
        }
      }
}

// ---------------------------------------------------------------------------
// K3/K4: triangular solve with an nb x nb diagonal block, on CW columns per
// workgroup: B[base:base+nb, cols] <- op(T)^{-1} B[base:base+nb, cols].
// op(T) is the stored row-major block (LOWER/UPPER part, UNIT diagonal or not)
// or, with CONJT, the conjugate transpose of the stored block.
// With MOVES the step's row moves are applied to the columns first (rows
// anywhere in the matrix; moved rows outside the block are written back).
// grid (ceil(ncols/CW), batch), block 256.  Substitution in LDS, row by row.
// ---------------------------------------------------------------------------
template <typename R, bool LOWER, bool UNIT, bool CONJT, bool MOVES, int CW>
__global__ __launch_bounds__(256) void k_trsm(const cx<R>* __restrict__ Tm, int64_t sT, int64_t ldt,
                                              cx<R>* __restrict__ Bm, int64_t sB, int64_t ldb, int ncols,
                                              int base, int nb, const int* __restrict__ moves, int64_t smv) {
  using T = cx<R>;
  __shared__ T Ts[NB_MAX][NB_MAX + 1];
  __shared__ T Bt[NB_MAX][CW];
  __shared__ T Mv[MOVES ? MOVE_CAP : 1][CW];
  const int bb = blockIdx.y;
  Tm += bb * sT;
  Bm += bb * sB;
  const int tid = threadIdx.x;
  const int cb = blockIdx.x * CW;
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e / nb, k = e % nb;
    T v;
    if (!CONJT) {
      v = Tm[(int64_t)i * ldt + k];
    } else {
      v = cconj(Tm[(int64_t)k * ldt + i]);
    }
    Ts[i][k] = v;
  }
  for (int e = tid; e < nb * CW; e += 256) {
    const int i = e / CW, c = e % CW;
    Bt[i][c] = (cb + c < ncols) ? Bm[(int64_t)(base + i) * ldb + cb + c] : czero<T>();
  }
  if (MOVES) {
    const int* mv = moves + bb * smv;
    const int cnt = mv[0];
    const int* dst = mv + 1;
    const int* src = mv + 1 + MOVE_CAP;
    for (int e = tid; e < cnt * CW; e += 256) {
      const int i = e / CW, c = e % CW;
      Mv[i][c] = (cb + c < ncols) ? Bm[(int64_t)src[i] * ldb + cb + c] : czero<T>();
    }
    __syncthreads();
    for (int e = tid; e < cnt * CW; e += 256) {
      const int i = e / CW, c = e % CW;
      const int d = dst[i];
      if (d >= base && d < base + nb)
        Bt[d - base][c] = Mv[i][c];
      else if (cb + c < ncols)
        Bm[(int64_t)d * ldb + cb + c] = Mv[i][c];
    }
  }
  __syncthreads();
  if (LOWER) {
    for (int k = 0; k < nb; ++k) {
      if (!UNIT) {
        if (tid < CW) Bt[k][tid] = cdiv(Bt[k][tid], Ts[k][k]);
        __syncthreads();
      }
      for (int e = tid; e < (nb - k - 1) * CW; e += 256) {
        const int i = k + 1 + e / CW, c = e % CW;
        Bt[i][c] = cfms(Bt[i][c], Ts[i][k], Bt[k][c]);
      }
      __syncthreads();
    }
  } else {
    for (int k = nb - 1; k >= 0; --k) {
      if (!UNIT) {
        if (tid < CW) Bt[k][tid] = cdiv(Bt[k][tid], Ts[k][k]);
        __syncthreads();
      }
      for (int e = tid; e < k * CW; e += 256) {
        const int i = e / CW, c = e % CW;
        Bt[i][c] = cfms(Bt[i][c], Ts[i][k], Bt[k][c]);
      }
      __syncthreads();
    }
  }
  for (int e = tid; e < nb * CW; e += 256) {
    const int i = e / CW, c = e % CW;
    if (cb + c < ncols) Bm[(int64_t)(base + i) * ldb + cb + c] = Bt[i][c];
  }
}

// ---------------------------------------------------------------------------
// Row moves of factorization steps [s_begin, s_end) applied to ncols columns:
// forward (P^T, steps in order, new[dst] = old[src]) or inverse (P, steps in
// reverse order, new[src] = old[dst]).  grid (ceil(ncols/CW), batch)
// ---------------------------------------------------------------------------
template <typename R, int CW>
__global__ __launch_bounds__(256) void k_moves(cx<R>* __restrict__ Bm, int64_t sB, int64_t ldb, int ncols,
                                               const int* __restrict__ moves, int64_t smv, int s_begin,
                                               int s_end, int inverse) {
  using T = cx<R>;
  __shared__ T Mv[MOVE_CAP][CW];
  const int bb = blockIdx.y;
  Bm += bb * sB;
  const int* mvb = moves + bb * smv;
  const int tid = threadIdx.x;
  const int cb = blockIdx.x * CW;
  const int ns = s_end - s_begin;
  for (int q = 0; q < ns; ++q) {
    const int step = inverse ? s_end - 1 - q : s_begin + q;
    const int* mv = mvb + (int64_t)step * MOVE_STRIDE;
    const int cnt = mv[0];
    const int* from = inverse ? mv + 1 : mv + 1 + MOVE_CAP;
    const int* to = inverse ? mv + 1 + MOVE_CAP : mv + 1;
    for (int e = tid; e < cnt * CW; e += 256) {
      const int i = e / CW, c = e % CW;
      if (cb + c < ncols) Mv[i][c] = Bm[(int64_t)from[i] * ldb + cb + c];
    }
    __syncthreads();
    for (int e = tid; e < cnt * CW; e += 256) {
      const int i = e / CW, c = e % CW;
      if (cb + c < ncols) Bm[(int64_t)to[i] * ldb + cb + c] = Mv[i][c];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Right-hand-side staging: nblk copies of V (column-major n x m, FP64) into the
// row-major solution array (npad x ldS, block b at columns [b*mp, b*mp+mp)),
// zero-padded; V == nullptr stages the identity.  grid-stride over npad*ldS.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_stage(cx<R>* __restrict__ X, int64_t ldS, int npad, int mp, int nblk,
                                               const double2* __restrict__ Vin, int64_t ldv, int n, int m) {
  const int64_t total = (int64_t)npad * ldS;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / ldS);
    const int jj = (int)(e % ldS);
    const int j = jj % mp;
    double2 v = czero<double2>();
    if (Vin) {
      if (i < n && j < m) v = Vin[i + (int64_t)j * ldv];
    } else if (i == j && i < n) {
      v.x = 1;
    }
    cx<R> o;
    o.x = (R)v.x;
    o.y = (R)v.y;
    X[e] = o;
  }
}

// ---------------------------------------------------------------------------
// K10 (thin V): X = sum_p (a_p Y_p + conj(a_p) Z_p), Y_p the solution for pole
// theta_p (block p) and Z_p the one for conj(theta_p) (block P+p), in FP64 in
// the fixed pair order (eq. equ:expAx with Remark rem:two_time_real_part).
// Output column-major n x m.  One thread per output element.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_accum_thin(const double2* __restrict__ Xs, int64_t ldS, int mp, int P,
                                                    const double2* __restrict__ a, int n, int m,
                                                    double2* __restrict__ out, int64_t ldx) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * m) return;
  const int i = (int)(e / m), j = (int)(e % m);
  const double2* row = Xs + (int64_t)i * ldS;
  double sr = 0, si = 0;
  for (int p = 0; p < P; ++p) {
    const double2 ap = a[p];
    const double2 y = row[p * mp + j];
    const double2 z = row[(P + p) * mp + j];
    sr += ap.x * y.x - ap.y * y.y + ap.x * z.x + ap.y * z.y;
    si += ap.x * y.y + ap.y * y.x + ap.x * z.y - ap.y * z.x;
  }
  double2 o;
  o.x = sr;
  o.y = si;
  out[i + (int64_t)j * ldx] = o;
}

// ---------------------------------------------------------------------------
// K10 (V = I): X = sum_p (a_p Y_p + (a_p Y_p)^H), Y_p = (tA + theta_p I)^{-1}
// (block p of the solution array, npad columns each): the conjugate pole's
// inverse is the adjoint of Y_p (eq. equ:ExpoMatRat with Remark
// rem:two_time_real_part).  32x32 output tiles through LDS; column-major out.
// grid (ceil(n/32), ceil(n/32)), block (32, 8)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_accum_full(const double2* __restrict__ Xs, int64_t ldS, int npad, int P,
                                                    const double2* __restrict__ a, int n,
                                                    double2* __restrict__ out, int64_t ldx) {
  __shared__ double2 t1[32][33];
  __shared__ double2 t2[32][33];
  const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
  const int tx = threadIdx.x, ty = threadIdx.y;
  double sr[4] = {0, 0, 0, 0}, si[4] = {0, 0, 0, 0};
  for (int p = 0; p < P; ++p) {
    const double2* Y = Xs + (int64_t)p * npad;
    __syncthreads();
    for (int q = 0; q < 4; ++q) {
      const int rr = ty + 8 * q;
      t1[rr][tx] = Y[(int64_t)(bi + rr) * ldS + bj + tx];  // (i, j) block
      t2[rr][tx] = Y[(int64_t)(bj + rr) * ldS + bi + tx];  // (j, i) block
    }
    __syncthreads();
    const double2 ap = a[p];
    for (int q = 0; q < 4; ++q) {
      const int jj = ty + 8 * q;
      // w1 = a Y[i][j], w2 = a Y[j][i] with identical rounding, so entry (j, i)
      // accumulates exactly the conjugate of entry (i, j): the output is
      // Hermitian bit for bit and its diagonal exactly real.
      const double2 y = t1[tx][jj];
      const double2 z = t2[jj][tx];
      const double w1x = fma(ap.x, y.x, -(ap.y * y.y)), w1y = fma(ap.x, y.y, ap.y * y.x);
      const double w2x = fma(ap.x, z.x, -(ap.y * z.y)), w2y = fma(ap.x, z.y, ap.y * z.x);
      sr[q] += w1x + w2x;
      si[q] += w1y - w2y;
    }
  }
  for (int q = 0; q < 4; ++q) {
    const int i = bi + tx, j = bj + ty + 8 * q;
    if (i < n && j < n) {
      double2 o;
      o.x = sr[q];
      o.y = si[q];
      out[i + (int64_t)j * ldx] = o;
    }
  }
}

// ---------------------------------------------------------------------------
// Mixed-precision helpers (refinement of every shifted solve in FP64).
// ---------------------------------------------------------------------------
template <typename RI, typename RO>
__global__ __launch_bounds__(256) void k_convert(const cx<RI>* __restrict__ in, cx<RO>* __restrict__ out,
                                                 int64_t count) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
    cx<RO> o;
    o.x = (RO)in[e].x;
    o.y = (RO)in[e].y;
    out[e] = o;
  }
}

// X64 += D32
__global__ __launch_bounds__(256) void k_add_correction(double2* __restrict__ X, const float2* __restrict__ D,
                                                        int64_t count) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x) {
    X[e].x += (double)D[e].x;
    X[e].y += (double)D[e].y;
  }
}

// Rres -= shift_b * X for block b (primal blocks theta_p, adjoint blocks conj(theta_p)).
__global__ __launch_bounds__(256) void k_shift_sub(double2* __restrict__ Rres, const double2* __restrict__ X,
                                                   int64_t ldS, int npad, int mp, int P,
                                                   const double2* __restrict__ theta) {
  const int64_t total = (int64_t)npad * ldS;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int blk = (int)((e % ldS) / mp);
    double2 th = theta[blk < P ? blk : blk - P];
    if (blk >= P) th.y = -th.y;
    const double2 x = X[e];
    Rres[e].x -= th.x * x.x - th.y * x.y;
    Rres[e].y -= th.x * x.y + th.y * x.x;
  }
}

}  // namespace expm

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
// Internal linkage: every translation unit that includes this file gets its own
// copies of the kernels it uses.
namespace {

// ---------------------------------------------------------------------------
// Stores one problem descriptor into device memory (the single-problem path
// when it replays a captured graph: the graph's kernels read the descriptor
// from memory, so new A, V, X and t need no change to the graph).
// grid 1, block 1
// ---------------------------------------------------------------------------
__global__ void k_put_desc(ProblemDesc* dst, ProblemDesc d) { *dst = d; }

// ---------------------------------------------------------------------------
// Pole and residue constants of one plan, passed by value (at most 32 pairs for
// the largest degree, 64), and their store into device memory.  Used where the
// workspace lives in the library's fixed device array and no host-to-device
// copy from caller memory is wanted.
// grid 1, block 64
// ---------------------------------------------------------------------------
struct PoleConsts {
  double2 theta[32], a[32];
};
__global__ void k_put_consts(double2* __restrict__ theta, double2* __restrict__ a, PoleConsts c, int P) {
  const int i = threadIdx.x;
  if (i < P) {
    theta[i] = c.theta[i];
    a[i] = c.a[i];
  }
}

// Fill of count ints with `value` (a kernel, not a memset node, so that a
// caller's stream capture records only kernels).  grid-stride.
__global__ __launch_bounds__(256) void k_fill(int* __restrict__ p, int64_t count, int value) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < count; e += (int64_t)gridDim.x * blockDim.x)
    p[e] = value;
}

// ---------------------------------------------------------------------------
// Per-problem status: *d.info = 2 if the result X (n x m, column-major) holds a
// non-finite value (non-finite input; a zero pivot cannot occur for finite
// Hermitian A, since |lambda + theta_k| >= |Im theta_k| > 0), else 1 if the
// refinement of one of its solves missed its tolerance (ir_nc[g] set), else 0.
// Problems without a status word are skipped.
// grid (G), block 256
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_status(const ProblemDesc* __restrict__ descs, ProblemDesc one,
                                                const int* __restrict__ ir_nc) {
  const ProblemDesc d = desc_of(descs, one, blockIdx.x);
  if (d.info == nullptr) return;
  int bad = 0;
  const int64_t count = (int64_t)d.n * d.m;
  for (int64_t e = threadIdx.x; e < count; e += 256) {
    const double2 v = d.X[(e % d.n) + (e / d.n) * d.ldx];
    bad |= !(isfinite(v.x) && isfinite(v.y));
  }
  bad = __syncthreads_or(bad);
  if (threadIdx.x == 0) *d.info = bad ? 2 : (ir_nc && ir_nc[blockIdx.x]) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// K1: form the shifted matrices  W_p = t*A + theta_p I  (paper Sec. 3,
// eqs. equ:ExpoMatRat and equ:expAx: one shifted matrix per pole; with the
// conjugate pairs of Remark rem:two_time_real_part one per pair suffices).
// A is column-major, lower (or, with d.upper, upper) triangle read; the
// Hermitian operand is built here so that W_p for conj(theta_p) would be
// exactly W_p^H.  The shift is added in
// FP64 before any rounding to the working type.  Optionally also writes
// Ah = t*A (full Hermitian, FP64, row-major) for the refinement residuals.
// grid (npad/32, npad/32), block (32, 8)
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_form(const ProblemDesc* __restrict__ descs, ProblemDesc one, int npad,
                                              const double2* __restrict__ theta, int P, cx<R>* __restrict__ Wb,
                                              int64_t wstride, int64_t ldw, double2* __restrict__ Ahb, int64_t ldh) {
  __shared__ double2 tile[32][33];
  const int g = blockIdx.z;
  const ProblemDesc d = desc_of(descs, one, g);
  const double2* A = d.A;
  const int64_t lda = d.lda;
  const int n = d.n;
  const double t = d.t;
  cx<R>* W = Wb + (int64_t)g * P * wstride;
  double2* Ah = Ahb ? Ahb + (int64_t)g * npad * ldh : nullptr;
  const int bi = blockIdx.y, bj = blockIdx.x;
  const int R0 = (bi > bj ? bi : bj) * 32, C0 = (bi < bj ? bi : bj) * 32;
  // tile[cc][x] = lower-triangle element (R0 + x, C0 + cc): read directly, or as
  // the conjugate of the upper element (C0 + cc, R0 + x), read along its column
  // and transposed through the tile
  for (int cc = threadIdx.y; cc < 32; cc += 8) {
    if (!d.upper) {
      const int r = R0 + threadIdx.x, c = C0 + cc;
      double2 v = czero<double2>();
      if (r < n && c < n) v = A[r + (int64_t)c * lda];
      if (d.real) v.y = 0;
      tile[cc][threadIdx.x] = v;
    } else {
      const int r = C0 + threadIdx.x, c = R0 + cc;
      double2 v = czero<double2>();
      if (r < n && c < n) v = cconj(A[r + (int64_t)c * lda]);
      if (d.real) v.y = 0;
      tile[threadIdx.x][cc] = v;
    }
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
          w.x += theta[p].x - d.c;
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
// IB columns [c0, c0+IB) over rows [c0, npad), one shifted matrix per
// workgroup.  The panel lives in registers: thread t holds the rows it loaded,
// c0 + t + PANEL_NT*s, for the whole panel.  A row interchange exchanges
// positions, not data: pos[s] is the row position the data in a[s] currently
// stand for, and the rows are written to their final positions when the panel
// is stored.  Per column (one barrier): every wave finds its candidate row
// (largest |Re|+|Im|, lowest position on ties) with DPP reductions and
// publishes value, position and the row's remaining columns in LDS; after the
// barrier every wave reduces the PANEL_NT/64 candidates the same way, reads
// the pivot row, exchanges the two positions and applies the rank-1 update in
// registers.  Every wave repeats the per-column bookkeeping (reductions, pivot
// reciprocal), so the workgroup is kept at 8 waves with more rows per thread
// rather than 16.  The panel is loaded and stored through LDS so that global
// accesses are coalesced.
// Then, inside the enclosing outer panel [j0, j0+nbo): the IB interchanges are
// applied to the other outer-panel columns and the IB x (rest) block of U is
// solved with the unit lower IB x IB factor.  On the last inner step the net
// row moves of the whole outer step are written for the later updates.
// grid (batch), block PANEL_NT
// ---------------------------------------------------------------------------
constexpr int PANEL_NT = 512;
constexpr int PANEL_NW = PANEL_NT / 64;

template <typename R, int IB>
struct PanelShared {
  R cand_v[2][PANEL_NW];
  int cand_i[2][PANEL_NW];
  cx<R> cand_row[2][PANEL_NW][IB];  // each wave's candidate row (columns C.. of step C)
  int piv[NB_MAX];
};

// Maximum of non-negative search values (or -1 for "no row"), over the wave and
// over each 16-lane row.  For FP32 the values are compared as signed integers:
// for floats >= 0 the bit patterns order like the values and -1.0f is negative,
// which saves the NaN canonicalisation a float maximum carries (no search value
// is NaN).
template <typename R>
__device__ __forceinline__ R search_wave_max(R x) {
  if constexpr (sizeof(R) == 4) {
    int v = __float_as_int(x);
    v = dpp_max_i32<0xB1, 0xF>(v);
    v = dpp_max_i32<0x4E, 0xF>(v);
    v = dpp_max_i32<0x141, 0xF>(v);
    v = dpp_max_i32<0x140, 0xF>(v);
    v = dpp_max_i32<0x142, 0xA>(v);
    v = dpp_max_i32<0x143, 0xC>(v);
    return __int_as_float(__builtin_amdgcn_readlane(v, 63));
  } else {
    return wave_max(x);
  }
}
template <typename R>
__device__ __forceinline__ R search_row16_max(R x) {
  if constexpr (sizeof(R) == 4) {
    int v = __float_as_int(x);
    v = dpp_max_i32<0xB1, 0xF>(v);
    v = dpp_max_i32<0x4E, 0xF>(v);
    v = dpp_max_i32<0x141, 0xF>(v);
    v = dpp_max_i32<0x140, 0xF>(v);
    return __int_as_float(v);
  } else {
    return row16_max(x);
  }
}

// LDS staging slot of element (row, col) of a PANEL_NT x IB block; the column is
// XOR-swizzled with the row so that one-row-per-lane reads spread over banks.
template <int IB>
__device__ __forceinline__ int stage_slot(int row, int col) {
  return row * IB + (col ^ (row & (IB - 1)));
}

// One column C of the inner panel.  Positions below gc = c0 + C belong to the
// earlier pivot rows; padding rows (past npad) carry position -1 and are never
// searched, updated or stored; every other row is active.  A NaN search value
// counts as 0, so some active row always wins (the lowest position among
// equals) and every pivot position stays inside the matrix.
template <typename R, int IB, int S, int C>
__device__ __forceinline__ void panel_column(cx<R> (&a)[S][IB], int (&pos)[S], PanelShared<R, IB>& sh, int c0,
                                             int j0, int tid) {
  if constexpr (C < IB) {
    using T = cx<R>;
    constexpr int NONE = 0x7fffffff;
    const int lane = tid & 63, wid = tid >> 6;
    const int gc = c0 + C;
    constexpr int buf = C & 1;
    // An active row of block s >= 1 still stands for the position it was loaded
    // at (only pivots leave, and they become inactive), so those rows are in
    // increasing position order and a strict comparison keeps the lowest
    // position among equal values; the row of block 0 may stand for a
    // position past them (a row displaced by a pivot) and takes the full rule.
    R bv = -1;
    int bi = NONE, bs = 0;
#pragma unroll
    for (int s = 1; s < S; ++s) {
      const R v = fmax(fabs(a[s][C].x) + fabs(a[s][C].y), (R)0);
      if (pos[s] >= gc && v > bv) {
        bv = v;
        bi = pos[s];
        bs = s;
      }
    }
    {
      const R v = fmax(fabs(a[0][C].x) + fabs(a[0][C].y), (R)0);
      if (pos[0] >= gc && (v > bv || (v == bv && pos[0] < bi))) {
        bv = v;
        bi = pos[0];
        bs = 0;
      }
    }
    // wave candidate: maximum value, then the lowest position among the lanes
    // holding it; cl is its lane and ws the block of that lane's row
    const R wv = search_wave_max(bv);
    const unsigned long long m = __ballot(bv == wv);
    int cl = __ffsll((long long)m) - 1;
    if (__popcll(m) != 1) {
      const int wmin = wave_min(bv == wv ? bi : NONE);
      cl = __ffsll((long long)__ballot(bv == wv && bi == wmin)) - 1;
    }
    const int wi = __builtin_amdgcn_readlane(bi, cl);
    const int ws = __builtin_amdgcn_readlane(bs, cl);
    if (lane == 0) {
      sh.cand_v[buf][wid] = wv;
      sh.cand_i[buf][wid] = wi;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (s == ws && lane == cl) {
#pragma unroll
        for (int cc = C; cc < IB; ++cc) sh.cand_row[buf][wid][cc] = a[s][cc];
      }
    }
    __syncthreads();
    // global pivot: each row of 16 lanes reduces the wave candidates (each
    // candidate held by 16 / PANEL_NW lanes of the row); lane l holds the
    // candidate of wave l % PANEL_NW, so the lowest lane holding the winner
    // is its wave
    const R cv = sh.cand_v[buf][lane % PANEL_NW];
    const int ci = sh.cand_i[buf][lane % PANEL_NW];
    const R gv = search_row16_max(cv);
    const int q = __builtin_amdgcn_readlane(row16_min(cv == gv ? ci : NONE), 0);
    const int pw = __ffsll((long long)__ballot(ci == q)) - 1;
    if (tid == 0) sh.piv[gc - j0] = q;
    // the part of the pivot row the update uses, read once into registers
    T pr[IB];
#pragma unroll
    for (int cc = C; cc < IB; ++cc) pr[cc] = sh.cand_row[buf][pw][cc];
    // interchange positions gc and q
#pragma unroll
    for (int s = 0; s < S; ++s) pos[s] = pos[s] == q ? gc : (pos[s] == gc ? q : pos[s]);
    const T inv = crecip_fast(pr[C]);
    // the rows below the pivot position
#pragma unroll
    for (int s = 0; s < S; ++s) {
      if (pos[s] > gc) {
        const T l = cmul(a[s][C], inv);
        a[s][C] = l;
#pragma unroll
        for (int cc = C + 1; cc < IB; ++cc) a[s][cc] = cfms(a[s][cc], l, pr[cc]);
      }
    }
    panel_column<R, IB, S, C + 1>(a, pos, sh, c0, j0, tid);
  }
}

template <typename R, int IB, int S>
__global__ __launch_bounds__(PANEL_NT) void k_panel(cx<R>* __restrict__ Wb, int64_t wstride, int64_t ld, int npad, int j0,
                                                int c0, int nbo, int* __restrict__ ipivb, int64_t pstride,
                                                int* __restrict__ movesb, int64_t mstride, int step, int last) {
  using T = cx<R>;
  __shared__ PanelShared<R, IB> sh;
  __shared__ T stage[PANEL_NT * IB];  // panel staging; reused as the row-move buffer
  __shared__ T Lib[IB][IB + 1];
  __shared__ int mv_dst[MOVE_CAP], mv_src[MOVE_CAP];
  __shared__ int mv_row[IB];
  __shared__ int mv_cnt;

  const int b = blockIdx.x;
  T* W = Wb + b * wstride;
  int* ipiv = ipivb + b * pstride;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;

  if (tid < c0 - j0) sh.piv[tid] = ipiv[j0 + tid];  // pivots of the earlier inner steps
  // all S*IB loads of the panel are issued before the first is used: element
  // q of block s is row rbase + (tid + PANEL_NT*q) / IB, column (tid + ...) % IB
  // (consecutive threads read consecutive columns of a row), held in a[s][q]
  // until the LDS round trip turns it into row-per-thread order
  // Addresses: a wave-uniform base (panel origin) plus one 32-bit byte offset
  // per lane; the per-element parts (q, s) are uniform multiples of the row
  // pitch.  Rows past npad read the panel origin instead (and are zeroed below).
  T a[S][IB];
  static_assert(PANEL_NT % IB == 0, "whole rows per pass");
  const char* pbase = (const char*)(W + (int64_t)c0 * ld + c0);
  const unsigned pitch = (unsigned)ld * (unsigned)sizeof(T);
  const unsigned lane_off = (unsigned)(tid / IB) * pitch + (unsigned)(tid % IB) * (unsigned)sizeof(T);
#pragma unroll
  for (int s = 0; s < S; ++s) {
#pragma unroll
    for (int q = 0; q < IB; ++q) {
      const int rr = PANEL_NT * s + (PANEL_NT / IB) * q;  // row offset of this pass (uniform)
      const bool ok = c0 + rr + tid / IB < npad;
      a[s][q] = *(const T*)(pbase + (ok ? lane_off + (unsigned)rr * pitch : 0u));
    }
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int rbase = c0 + PANEL_NT * s;
    const int nr = npad - rbase < PANEL_NT ? npad - rbase : PANEL_NT;
#pragma unroll
    for (int q = 0; q < IB; ++q) {
      const int e = tid + PANEL_NT * q;
      stage[stage_slot<IB>(e / IB, e % IB)] = a[s][q];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < IB; ++c) a[s][c] = tid < nr ? stage[stage_slot<IB>(tid, c)] : czero<T>();
    __syncthreads();
  }
  int pos[S];
#pragma unroll
  for (int s = 0; s < S; ++s) pos[s] = c0 + tid + PANEL_NT * s < npad ? c0 + tid + PANEL_NT * s : -1;
  panel_column<R, IB, S, 0>(a, pos, sh, c0, j0, tid);

  // store: block sb of positions gathers the rows that now stand for them.
  // Only two kinds of row change blocks: the pivot rows (to positions
  // [c0, c0+IB) of block 0) and the rows they displaced, which all started at
  // those positions (block 0 of wave 0, lanes below IB).
#pragma unroll
  for (int sb = 0; sb < S; ++sb) {
    const int rbase = c0 + PANEL_NT * sb;
    {
      const int r = pos[sb] - rbase;
      if (r >= 0 && r < PANEL_NT) {
#pragma unroll
        for (int c = 0; c < IB; ++c) stage[stage_slot<IB>(r, c)] = a[sb][c];
      }
    }
    if (sb == 0) {
#pragma unroll
      for (int s = 1; s < S; ++s) {
        if (pos[s] >= c0 && pos[s] < c0 + IB) {
#pragma unroll
          for (int c = 0; c < IB; ++c) stage[stage_slot<IB>(pos[s] - c0, c)] = a[s][c];
        }
      }
    } else if (wid == 0) {
      const int r = pos[0] - rbase;
      if (r >= 0 && r < PANEL_NT) {
#pragma unroll
        for (int c = 0; c < IB; ++c) stage[stage_slot<IB>(r, c)] = a[0][c];
      }
    }
    __syncthreads();
    if (sb == 0 && tid < IB) {
#pragma unroll
      for (int c = 0; c < IB; ++c) Lib[tid][c] = stage[stage_slot<IB>(tid, c)];  // rows c0..c0+IB of the factors
    }
#pragma unroll
    for (int q = 0; q < IB; ++q) {
      const int e = tid + PANEL_NT * q;
      const int rr = PANEL_NT * sb + (PANEL_NT / IB) * q;
      if (c0 + rr + tid / IB < npad)
        *(T*)((char*)pbase + lane_off + (unsigned)rr * pitch) = stage[stage_slot<IB>(e / IB, e % IB)];
    }
    __syncthreads();
  }
  if (tid < IB) ipiv[c0 + tid] = sh.piv[c0 - j0 + tid];
  if (wid == 0) {
    // mv_row: for each row of the U block, the move that fills it (-1: none)
    const int cnt = composite_moves(sh.piv + (c0 - j0), IB, c0, mv_dst, mv_src, mv_row);
    if (lane == 0) mv_cnt = cnt;
  }
  __syncthreads();

  // ---- interchanges on the other columns of the outer panel, then U block --
  // The moved values and the U block's rows (as they stand before the
  // interchanges) are read together; the U block takes the moved value where
  // a move fills one of its rows and writes all IB of its rows itself, so the
  // interchanges skip those rows of the right columns.
  T* mvbuf = stage;  // [2*IB][NB_MAX]
  const int nleft = c0 - j0, nright = j0 + nbo - c0 - IB, nother = nleft + nright;
  const int cnt = mv_cnt;
  // at most 2*IB moves over fewer than NB_MAX columns: MV_IT passes cover them
  constexpr int MV_IT = (2 * IB * NB_MAX + PANEL_NT - 1) / PANEL_NT;
  // (FP64: unconditional loads, the unused ones of the matrix's first element;
  // guarded ones put the values in scratch memory there and serialize them)
  T mvv[MV_IT];
#pragma unroll
  for (int it = 0; it < MV_IT; ++it) {
    const int e = tid + PANEL_NT * it;
    const bool ok = e < cnt * nother;
    if constexpr (sizeof(R) == 8) {
      const int i = ok ? e / nother : 0, cc = ok ? e % nother : 0;
      const int col = cc < nleft ? j0 + cc : c0 + IB + (cc - nleft);
      mvv[it] = W[ok ? (int64_t)mv_src[i] * ld + col : 0];
    } else if (ok) {
      const int i = e / nother, cc = e % nother;
      const int col = cc < nleft ? j0 + cc : c0 + IB + (cc - nleft);
      mvv[it] = W[(int64_t)mv_src[i] * ld + col];
    }
  }
  T x[IB];
  if (tid < nright) {
#pragma unroll
    for (int i = 0; i < IB; ++i) x[i] = W[(int64_t)(c0 + i) * ld + c0 + IB + tid];
  }
#pragma unroll
  for (int it = 0; it < MV_IT; ++it) {
    const int e = tid + PANEL_NT * it;
    if (e < cnt * nother) mvbuf[(e / nother) * NB_MAX + e % nother] = mvv[it];
  }
  __syncthreads();
  for (int e = tid; e < cnt * nother; e += PANEL_NT) {
    const int i = e / nother, cc = e % nother;
    const int col = cc < nleft ? j0 + cc : c0 + IB + (cc - nleft);
    const int dst = mv_dst[i];
    if (cc < nleft || dst >= c0 + IB) W[(int64_t)dst * ld + col] = mvbuf[i * NB_MAX + cc];
  }
  if (tid < nright) {
    const int col = c0 + IB + tid;
#pragma unroll
    for (int i = 0; i < IB; ++i) {
      if constexpr (sizeof(R) == 8) {
        // (these threads are all in wave 0, so the move index is wave-uniform;
        // a select of the two values puts x in scratch memory in FP64)
        const int sl = __builtin_amdgcn_readfirstlane(mv_row[i]);
        if (sl >= 0) x[i] = mvbuf[sl * NB_MAX + nleft + tid];
      } else {
        const int sl = mv_row[i];
        const T v = mvbuf[(sl < 0 ? 0 : sl) * NB_MAX + nleft + tid];
        x[i] = sl >= 0 ? v : x[i];
      }
    }
#pragma unroll
    for (int i = 1; i < IB; ++i)
#pragma unroll
      for (int k = 0; k < i; ++k) x[i] = cfms(x[i], Lib[i][k], x[k]);
#pragma unroll
    for (int i = 0; i < IB; ++i) W[(int64_t)(c0 + i) * ld + col] = x[i];
  }
  if (last && wid == 0) {
    // net row moves of the whole outer step
    int* mv = movesb + b * mstride + (int64_t)step * MOVE_STRIDE;
    const int cnt2 = composite_moves(sh.piv, nbo, j0, mv + 1, mv + 1 + MOVE_CAP);
    if (lane == 0) mv[0] = cnt2;
  }
}

// ---------------------------------------------------------------------------
// Inverses of the nb x nb diagonal blocks of the LU factors: L11^{-1} (unit
// lower) and U11^{-1} (upper), so that the triangular solves of the update and
// the sweeps run as matrix-core products.  One wave per group of four columns
// of an inverse: lane i holds row i; forward (L) or backward (U) substitution
// with the current pivot value broadcast by readlane, the four columns carried
// together to overlap their dependency chains.  A workgroup of BIW waves
// loads the diagonal block into LDS once (coalesced rows) and covers 4*BIW
// columns; the result is staged back through LDS and written as whole rows.
// BIW = 4 spreads a launch with few blocks over more CUs; BIW = 16 (one
// workgroup per block) loads each block once and keeps more waves per CU when
// a launch has many blocks.  Every column is computed the same way in both.
// grid (16/BIW * nsteps_range * (1 or 2), batch), block 64*BIW;
// blockIdx.x encodes (step, L or U, group of 4*BIW columns).
// ---------------------------------------------------------------------------
template <typename R, int BIW>
__device__ __forceinline__ void block_inverse_body(int g, int b, const cx<R>* __restrict__ Wb, int64_t wstride,
                                                   int64_t ld, int step0, int which, cx<R>* __restrict__ dinvb,
                                                   int64_t dstride, cx<R> (*D)[NB_MAX + 1], cx<R>* rdiag) {
  using T = cx<R>;
  constexpr int NB = NB_MAX, NT = 64 * BIW, GROUPS = 16 / BIW;
  static_assert(16 % BIW == 0, "whole column groups");
  const int nmat = which == 2 ? 2 : 1;  // which: 0 = L only, 1 = U only, 2 = both
  const int wg = g % GROUPS;
  const int mat = (g / GROUPS) % nmat;
  const int step = step0 + g / (GROUPS * nmat);
  const bool upper = which == 1 || (which == 2 && mat == 1);
  const T* W = Wb + b * wstride;
  const int j0 = step * NB;
  const int tid = threadIdx.x, lane = tid & 63;
  const int cgrp = wg * BIW + (tid >> 6);  // this wave's four columns: 4*cgrp ..
  // the 64 x 64 diagonal block into LDS: every load issued before the first
  // store (consecutive threads read consecutive columns of a row)
  {
    constexpr int PER = NB * NB / NT;
    T v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + NT * u;
      v[u] = W[(int64_t)(j0 + e / NB) * ld + j0 + e % NB];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + NT * u;
      D[e / NB][e % NB] = v[u];
    }
  }
  __syncthreads();
  if (upper && tid < NB) rdiag[tid] = crecip(D[tid][tid]);
  __syncthreads();
  T one = czero<T>();
  one.x = 1;
  const int i = lane;
  T x[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) x[q] = (i == cgrp * 4 + q) ? one : czero<T>();
  if (!upper) {
    const int cmin = cgrp * 4;
    for (int k = cmin; k < NB - 1; ++k) {
      const T lik = D[i][k];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const T xk = lane_bcast2(x[q], k);
        if (i > k) x[q] = cfms(x[q], lik, xk);
      }
    }
  } else {
    const int cmax = cgrp * 4 + 3;
    for (int k = cmax; k >= 0; --k) {
      const T uik = D[i][k];
      const T rk = rdiag[k];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (i == k) x[q] = cmul(x[q], rk);
        const T xk = lane_bcast2(x[q], k);
        if (i < k) x[q] = cfms(x[q], uik, xk);
      }
    }
  }
  __syncthreads();  // every wave is done reading the block: D takes the result
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = cgrp * 4 + q;
    const bool keep = upper ? (i <= c) : (i >= c);
    D[i][c] = keep ? x[q] : czero<T>();
  }
  __syncthreads();
  // the workgroup's 4*BIW columns of every row, written as row segments
  T* out = dinvb + b * dstride + (int64_t)step * 2 * NB * NB + (upper ? NB * NB : 0);
  constexpr int CW = 4 * BIW;
#pragma unroll
  for (int u = 0; u < NB * CW / NT; ++u) {
    const int e = tid + NT * u;
    const int r = e / CW, c = wg * CW + e % CW;
    out[r * NB + c] = D[r][c];
  }
}

template <typename R, int BIW>
__global__ __launch_bounds__(64 * BIW) void k_block_inverse(const cx<R>* __restrict__ Wb, int64_t wstride,
                                                                 int64_t ld, int step0, int which,
                                                                 cx<R>* __restrict__ dinvb, int64_t dstride) {
  __shared__ cx<R> D[NB_MAX][NB_MAX + 1];
  __shared__ cx<R> rdiag[NB_MAX];
  block_inverse_body<R, BIW>(blockIdx.x, blockIdx.y, Wb, wstride, ld, step0, which, dinvb, dstride, D, rdiag);
}

// ---------------------------------------------------------------------------
// K5: complex matrix products on the matrix cores, batched over blockIdx.y:
//   MODE 0:  C -= op(A) B        MODE 1:  C = op(A) B
// op(A) = A (row-major M x K) or, with conj, the conjugate transpose of a
// row-major K x M array.  blockIdx.y = g*ks + s: product g of the batch, K
// slice s of ks (split K: slice s starts at A + s*kA, B + s*kB and writes
// C + s*kC, so each slice's partial product lands in its own array).  Products
// g < split use operand a0 (at a0.p + g*a0.stride), the others a1 (at a1.p +
// (g-split)*a1.stride), so a primal and an adjoint sweep share one launch.
// B row-major K x N, C row-major M x N.
// MODE 1 may overwrite B in place when one row tile covers M (BM >= M): every
// workgroup reads all of its B columns before writing them.
// Complex products from real 16x16x4 products: the K dimension is interleaved
// (real index 2k = real part, 2k+1 = imaginary part), so with b = (Re B, Im B)
// per k, Re C uses a = (Re A, -Im A) and Im C uses a = (Im A, Re A): two real
// products per 16x16 complex block and pair of k, B operand shared.
// Tiles BM x BN per 256-thread workgroup, waves WGM x WGN, K staged through LDS
// in chunks of 16.
// ---------------------------------------------------------------------------
struct KSplit {
  int ks;             // K slices per product (1: no split)
  int64_t kA, kB, kC;  // element offsets of slice s: A + s*kA, B + s*kB, C + s*kC
};

template <typename R>
struct GemmOperand {
  const cx<R>* p;
  int64_t stride, ld;
  int conj;
};

// Waves per SIMD the register allocation of k_gemm is held to (the LDS of a
// 64 x 64 tile allows four workgroups per CU).  Unconstrained, the FP32 kernel
// takes 132 registers and runs three waves per SIMD.  Tiles of twice the area
// hold twice the accumulators and are given half the waves.
constexpr int GEMM_WAVES_F32 = 4, GEMM_WAVES_F64 = 2;
template <typename R, int BM, int BN>
constexpr int gemm_waves() {
  return (sizeof(R) == 4 ? GEMM_WAVES_F32 : GEMM_WAVES_F64) / (BM * BN > 64 * 64 ? 2 : 1);
}

// TAG 1 (the LU trailing update) and TAG 2 (the other products with whole
// tiles: the narrow K = 64 LU updates, U12 = L11^-1 A12, the refinement product
// and the block products of wide solves) are instantiations
// compiled for whole tiles and chunks (M a multiple of BM, N of BN, K of 16: no
// bounds checks or zero scaling) and an operand that is never conjugated, which
// keeps the operand fetch free of branches; separate instantiations so kernel
// traces and counters tell them apart.  The launcher uses them only for shapes
// that satisfy this.
template <typename R, int MODE, int BM, int BN, int WGM, int WGN, int TAG>
__device__ __forceinline__ void gemm_block(int M, int N, int K, GemmOperand<R> a0, GemmOperand<R> a1, int split,
                                           const cx<R>* B, int64_t sB, int64_t ldb, cx<R>* C, int64_t sC,
                                           int64_t ldc, KSplit ksp) {
  using T = cx<R>;
  using MF = Mfma<R>;
  using V = typename MF::V;
  constexpr int KC = 16;
  constexpr bool FULL = TAG >= 1;  // whole tiles and chunks, no conjugation (checked by the launcher)
  constexpr int WM = BM / WGM, WN = BN / WGN, MI = WM / 16, NJ = WN / 16;
  constexpr int AE = BM * KC / 256, BE = KC * BN / 256;  // chunk elements per thread
  static_assert(WGM * WGN == 4, "four waves");
  static_assert(AE >= 1 && BE >= 1, "tile too small");
  __shared__ T As[2][BM][KC + 1];
  __shared__ T Bs[2][KC][BN + 1];

  const int tiles_m = (M + BM - 1) / BM;
  const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
  const int bb = (int)blockIdx.y / ksp.ks, ks = (int)blockIdx.y % ksp.ks;
  const bool second = bb >= split;
  const GemmOperand<R> op = second ? a1 : a0;
  const T* A = op.p + (second ? bb - split : bb) * op.stride + ks * ksp.kA;
  const int64_t lda = op.ld;
  const bool conj = !FULL && op.conj != 0;
  B += bb * sB + ks * ksp.kB;
  C += bb * sC + ks * ksp.kC;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm0 = (w / WGN) * WM, wn0 = (w % WGN) * WN;
  const int r16 = lane & 15, kq = lane >> 4;
  const int m0 = tm * BM, n0 = tn * BN;

  // the products are summed on their own and subtracted from C once, in the
  // epilogue (MODE 0), so C's magnitude does not enter every rounding step.
  // Each complex product is formed from three real ones (Gauss: T1 = Re a Re b,
  // T2 = Im a Im b, T3 = (Re a + Im a)(Re b + Im b); Re = T1 - T2, Im = T3 - T1 - T2),
  // a quarter fewer matrix-core products than the four of the plain form.  Its
  // bound is normwise of the same order, componentwise weaker in Im; the errors of
  // the method are set by the cancellation in the pole sum, not by this rounding.
  // Every instantiation does the same, so all tile shapes give the same bits.
  V accR[MI][NJ], accI[MI][NJ], accS[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      accR[i][j] = V{0, 0, 0, 0};
      accI[i][j] = V{0, 0, 0, 0};
      accS[i][j] = V{0, 0, 0, 0};
    }

  // one K chunk of A (op applied, conjugated if needed) and B into registers.
  // Branch-free: out-of-range elements load from the operand's first element and
  // are scaled by zero when stashed (a multiply, not a select, so every load of a
  // chunk stays unconditional and in flight during the products of the current
  // chunk; the scaling is consumed only after them).
  T ra[AE], rb[BE];
  R fa[AE], fb[BE];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < AE; ++q) {
      const int e = tid + 256 * q;
      const int i = conj ? e % BM : e / KC, k = conj ? e / BM : e % KC;
      const bool ok = FULL || (m0 + i < M && k0 + k < K);
      const int64_t idx = !ok ? 0 : conj ? (int64_t)(k0 + k) * lda + m0 + i : (int64_t)(m0 + i) * lda + k0 + k;
      ra[q] = A[idx];
      fa[q] = ok ? R(1) : R(0);
    }
#pragma unroll
    for (int q = 0; q < BE; ++q) {
      const int e = tid + 256 * q;
      const int j = e % BN, k = e / BN;
      const bool ok = FULL || (n0 + j < N && k0 + k < K);
      rb[q] = B[ok ? (int64_t)(k0 + k) * ldb + n0 + j : 0];
      fb[q] = ok ? R(1) : R(0);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < AE; ++q) {
      const int e = tid + 256 * q;
      T v;
      v.x = FULL ? ra[q].x : ra[q].x * fa[q];
      v.y = FULL ? ra[q].y : (conj ? -ra[q].y : ra[q].y) * fa[q];
      if (!conj)
        As[buf][e / KC][e % KC] = v;
      else
        As[buf][e % BM][e / BM] = v;
    }
#pragma unroll
    for (int q = 0; q < BE; ++q) {
      const int e = tid + 256 * q;
      T v;
      v.x = FULL ? rb[q].x : rb[q].x * fb[q];
      v.y = FULL ? rb[q].y : rb[q].y * fb[q];
      Bs[buf][e / BN][e % BN] = v;
    }
  };

  const int nchunks = (K + KC - 1) / KC;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int ch = 0; ch < nchunks; ++ch) {
    const int cur = ch & 1;
    if (ch + 1 < nchunks) fetch((ch + 1) * KC);  // in flight during the products below
    {
      // four complex k per matrix-core step: lane (r16, kq) gives A[row r16][k kq]
      // and B[k kq][column r16]; accR, accI, accS collect T1, T2, T3
#pragma unroll
      for (int k4 = 0; k4 < KC / 4; ++k4) {
        const int kc = 4 * k4 + kq;
        R a1[MI], a2[MI], a3[MI], b1[NJ], b2[NJ], b3[NJ];
#pragma unroll
        for (int i = 0; i < MI; ++i) {
          const T av = As[cur][wm0 + i * 16 + r16][kc];
          a1[i] = av.x;
          a2[i] = av.y;
          a3[i] = av.x + av.y;
        }
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const T bv = Bs[cur][kc][wn0 + j * 16 + r16];
          b1[j] = bv.x;
          b2[j] = bv.y;
          b3[j] = bv.x + bv.y;
        }
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            accR[i][j] = MF::run(a1[i], b1[j], accR[i][j]);
            accI[i][j] = MF::run(a2[i], b2[j], accI[i][j]);
            accS[i][j] = MF::run(a3[i], b3[j], accS[i][j]);
          }
      }
    }
    if (ch + 1 < nchunks) stash(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const V t1 = accR[i][j], t2 = accI[i][j];
      accR[i][j] = t1 - t2;
      accI[i][j] = accS[i][j] - t1 - t2;
    }
  // epilogue: all C loads (clamped in range) first, then the guarded stores
  T cold[MI][NJ][4];
  if constexpr (MODE == 0) {
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm0 + i * 16 + MF::row(kq, r);
          const int col = n0 + wn0 + j * 16 + r16;
          const bool ok = FULL || (row < M && col < N);
          cold[i][j][r] = C[ok ? (int64_t)row * ldc + col : 0];
        }
  }
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm0 + i * 16 + MF::row(kq, r);
        const int col = n0 + wn0 + j * 16 + r16;
        T c;
        if constexpr (MODE == 0) {
          c = cold[i][j][r];
          c.x -= accR[i][j][r];
          c.y -= accI[i][j][r];
        } else {
          c.x = accR[i][j][r];
          c.y = accI[i][j][r];
        }
        if (FULL || (row < M && col < N)) C[(int64_t)row * ldc + col] = c;
      }
}

template <typename R, int MODE, int BM, int BN, int WGM, int WGN, int TAG = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(gemm_waves<R, BM, BN>()))) void k_gemm(
    int M, int N, int K, GemmOperand<R> a0, GemmOperand<R> a1, int split, const cx<R>* B, int64_t sB, int64_t ldb,
    cx<R>* C, int64_t sC, int64_t ldc, KSplit ksp) {
  gemm_block<R, MODE, BM, BN, WGM, WGN, TAG>(M, N, K, a0, a1, split, B, sB, ldb, C, sC, ldc, ksp);
}

// The same product, doing nothing when *gate == 0: the refinement sweeps after
// every solve of the launch has converged.
template <typename R, int MODE, int BM, int BN, int WGM, int WGN, int TAG = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(gemm_waves<R, BM, BN>()))) void k_gemm_gated(
    const int* __restrict__ gate, int M, int N, int K, GemmOperand<R> a0, GemmOperand<R> a1, int split,
    const cx<R>* B, int64_t sB, int64_t ldb, cx<R>* C, int64_t sC, int64_t ldc, KSplit ksp) {
  if (*gate == 0) return;
  gemm_block<R, MODE, BM, BN, WGM, WGN, TAG>(M, N, K, a0, a1, split, B, sB, ldb, C, sC, ldc, ksp);
}

// ---------------------------------------------------------------------------
// A whole block triangular sweep on thin right-hand sides in ONE launch.
// The right-hand sides are split into chains of 16 columns: chain c is
// columns [c16*16, c16*16+16) of pole block bb = c / cpb (cpb = 16-column
// chains per block), c16 = c % cpb, i.e. X + bb*sX + c16*16.  For row tile I
// (64 rows; tiles visited in sweep order, I = q forward or nsteps-1-q backward):
//   acc = sum over the tiles J before I in sweep order of A_IJ x_J
//   x_I = D_I (b_I - acc)       written over b_I in X
// D_I is the inverse of the diagonal block (or its conjugate transpose), A_IJ
// the off-diagonal block W[I rows][J cols] or, with conj, the conjugate
// transpose of W[J rows][I cols].  Blocks bb < split use operands *0, the
// others *1.
// Scheduling: a workgroup takes a ticket from ctl[SW_TICKET] when it starts;
// ticket t = q*nchain + c handles tile position q of chain c.  Its waits are on
// x_J of the same chain at positions < q, i.e. on smaller tickets, which were
// taken by workgroups already running: every wait ends.  x_J is announced by
// flags[(c*nsteps + J) * FLAG_STRIDE] == epoch, where the launch's epoch is one
// more than ctl[SW_EPOCH].  The workgroup that finishes last (ctl[SW_DONE]
// counts them) resets the ticket and finish counters and stores the epoch, so
// the next launch on the stream starts from ticket 0 with a new epoch: no
// launch argument changes between sweeps, and a captured graph replays them.
// Each wait is also capped; a capped wait records 1 in ctl[SW_STATUS] and the
// sweep result is then invalid.
// grid (nchain * nsteps), block 256: wave w owns rows 16w..16w+15 of the tile.
// ---------------------------------------------------------------------------
template <typename R>
struct SweepOperand {
  const cx<R>* p;
  int64_t stride, ld;
  int conj;
};

constexpr int SWEEP_SPIN_CAP = 1 << 20;
constexpr int FLAG_STRIDE = 32;  // one 128-byte line per ready flag
// words of the sweep control line (the first FLAG_STRIDE ints of the plan's
// sweep area; the ready flags follow it)
constexpr int SW_TICKET = 0, SW_STATUS = 1, SW_DONE = 2, SW_EPOCH = 3;

// eight consecutive complex values from a 16-byte aligned address
template <typename T>
__device__ __forceinline__ void load8(const T* p, T* a) {
  if constexpr (sizeof(T) == 8) {
    const float4* q = (const float4*)p;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float4 v = q[u];
      a[2 * u].x = v.x;
      a[2 * u].y = v.y;
      a[2 * u + 1].x = v.z;
      a[2 * u + 1].y = v.w;
    }
  } else {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = p[u];
  }
}

// Element at a byte offset from a wave-uniform base (offsets within one 64-row
// block always fit 32 bits), so loads take the scalar-base + 32-bit offset form.
template <typename T>
__device__ __forceinline__ const T& at_bytes(const T* base, unsigned off) {
  return *(const T*)((const char*)base + off);
}

// One complex MAC block for the wave's 16 x 16 output: 8 consecutive complex k
// of the lane's half (see below), a[u] = Blk(row, k), bv[u] = B(k, column).
template <typename R>
__device__ __forceinline__ void mac8(const cx<R>* a, const cx<R>* bv, bool odd, typename Mfma<R>::V& accR,
                                     typename Mfma<R>::V& accI) {
  using MF = Mfma<R>;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const R bR = odd ? bv[u].y : bv[u].x;
    accR = MF::run(odd ? -a[u].y : a[u].x, bR, accR);
    accI = MF::run(odd ? a[u].x : a[u].y, bR, accI);
  }
}

// Eight elements of the wave's 16 x 64 slice of a 64 x 64 block, in the
// product layout: lane (r16, kq) gets Blk(row0 + r16, 32h + k8 + u), u = 0..7,
// h = kq >> 1.  Each lane walks 32 consecutive k over the four chunks, so a
// row-major block is read with 16-byte loads along its rows.  Blk(i, k) =
// p[i*ld + k], or conj(p[k*ld + i]) with CONJ.  The base pointer is
// wave-uniform and all offsets inside one 64-row block fit 32 bits.
template <typename R, bool CONJ>
__device__ __forceinline__ void load_chunk(const cx<R>* p, int64_t ld, int row0, int k8, cx<R>* a) {
  using T = cx<R>;
  const int lane = threadIdx.x & 63;
  const int r16 = lane & 15, h = (lane >> 4) >> 1;
  const unsigned e = sizeof(T), lde = (unsigned)ld * e;
  const char* pb = (const char*)p;
  if constexpr (CONJ) {
    const unsigned off = (32u * h + k8) * lde + (unsigned)(row0 + r16) * e;
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] = cconj(*(const T*)(pb + off + u * lde));
  } else {
    load8((const T*)(pb + (unsigned)(row0 + r16) * lde + (32u * h + k8) * e), a);
  }
}

// Wait until the chain's flag for block J carries this launch's epoch (one
// wave polls, then the workgroup is released by a barrier).  Capped; a failed
// wait anywhere ends every later wait at once.
__device__ __forceinline__ void chain_wait(const int* flag, int epoch, int* status) {
  if ((threadIdx.x >> 6) == 0) {
    int spins = 0;
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
      __builtin_amdgcn_s_sleep(2);
      ++spins;
      if ((spins & 127) == 0 && __hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
      if (spins > SWEEP_SPIN_CAP) {
        atomicOr(status, 1);
        break;
      }
    }
  }
  __syncthreads();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

// x_J (64 rows x 16 columns at x, row pitch ldx) into LDS with coherent 16-byte
// loads, one pass over the block by the whole workgroup (256 threads)
template <typename R>
__device__ __forceinline__ void chain_fill(const cx<R>* x, int64_t ldx, cx<R> (*Xs)[17]) {
  using T = cx<R>;
  constexpr int PER_ROW = 16 * sizeof(T) / 16;  // 16-byte pieces per row
  constexpr int PIECES = 64 * PER_ROW / 256;    // per thread
  const unsigned pitch = (unsigned)ldx * sizeof(T);
  const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(x, 64u * pitch);
  const int tid = threadIdx.x;
  u32x4 v[PIECES];
#pragma unroll
  for (int q = 0; q < PIECES; ++q) {
    const int id = tid + 256 * q, row = id / PER_ROW, seg = id % PER_ROW;
    v[q] = coherent_load16(rs, (unsigned)row * pitch + (unsigned)seg * 16u);
  }
#pragma unroll
  for (int q = 0; q < PIECES; ++q) {
    const int id = tid + 256 * q, row = id / PER_ROW, seg = id % PER_ROW;
    if constexpr (sizeof(T) == 8) {
      T p0, p1;
      p0.x = __uint_as_float(v[q][0]);
      p0.y = __uint_as_float(v[q][1]);
      p1.x = __uint_as_float(v[q][2]);
      p1.y = __uint_as_float(v[q][3]);
      Xs[row][2 * seg] = p0;
      Xs[row][2 * seg + 1] = p1;
    } else {
      T p0;
      p0.x = __longlong_as_double(((long long)v[q][1] << 32) | v[q][0]);
      p0.y = __longlong_as_double(((long long)v[q][3] << 32) | v[q][2]);
      Xs[row][seg] = p0;
    }
  }
}

// The 64 x 16 block in Xs to x (row pitch ldx) with coherent 16-byte stores
template <typename R>
__device__ __forceinline__ void chain_publish(cx<R> (*Xs)[17], cx<R>* x, int64_t ldx) {
  using T = cx<R>;
  constexpr int PER_ROW = 16 * sizeof(T) / 16;
  constexpr int PIECES = 64 * PER_ROW / 256;
  const unsigned pitch = (unsigned)ldx * sizeof(T);
  const __amdgpu_buffer_rsrc_t rs = buffer_rsrc(x, 64u * pitch);
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < PIECES; ++q) {
    const int id = tid + 256 * q, row = id / PER_ROW, seg = id % PER_ROW;
    u32x4 v;
    if constexpr (sizeof(T) == 8) {
      const T p0 = Xs[row][2 * seg], p1 = Xs[row][2 * seg + 1];
      v[0] = __float_as_uint(p0.x);
      v[1] = __float_as_uint(p0.y);
      v[2] = __float_as_uint(p1.x);
      v[3] = __float_as_uint(p1.y);
    } else {
      const T p0 = Xs[row][seg];
      const unsigned long long a = (unsigned long long)__double_as_longlong(p0.x);
      const unsigned long long c = (unsigned long long)__double_as_longlong(p0.y);
      v[0] = (unsigned)a;
      v[1] = (unsigned)(a >> 32);
      v[2] = (unsigned)c;
      v[3] = (unsigned)(c >> 32);
    }
    coherent_store16(v, rs, (unsigned)row * pitch + (unsigned)seg * 16u);
  }
}

// acc = sum over the blocks J before I in sweep order of A_IJ x_J.  x_J is
// brought into LDS once per workgroup after its flag is seen.  FP32 slices are
// loaded before each wait (their loads overlap it); FP64 slices chunk by chunk
// after it, which keeps the registers for three workgroups per CU.
// Without WAIT (one workgroup walks the whole chain and wrote every x_J
// itself) a barrier replaces the wait: the previous block's LDS reads end
// before x_J is filled in.
template <typename R, bool CONJ, bool WAIT>
__device__ __forceinline__ void chain_accumulate(int q, int I, int fwd, int nsteps, const cx<R>* W, int64_t ld,
                                                 const cx<R>* Xc, int64_t ldx, int row0, const int* fl, int epoch,
                                                 int* status, cx<R> (*Xs)[17], typename Mfma<R>::V& accR,
                                                 typename Mfma<R>::V& accI) {
  using T = cx<R>;
  constexpr int NB = NB_MAX;
  const int lane = threadIdx.x & 63;
  const int r16 = lane & 15, h = (lane >> 4) >> 1;
  const bool odd = (lane >> 4) & 1;
  for (int qq = 0; qq < q; ++qq) {
    const int J = fwd ? qq : nsteps - 1 - qq;
    const T* Ablk = CONJ ? W + (int64_t)(J * NB) * ld + I * NB : W + (int64_t)(I * NB) * ld + J * NB;
    if constexpr (sizeof(R) == 4) {
      T a[32];
#pragma unroll
      for (int k8 = 0; k8 < 32; k8 += 8) load_chunk<R, CONJ>(Ablk, ld, row0, k8, a + k8);
      if constexpr (WAIT)
        chain_wait(fl + J * FLAG_STRIDE, epoch, status);
      else
        __syncthreads();
      chain_fill<R>(Xc + (int64_t)(J * NB) * ldx, ldx, Xs);
      __syncthreads();
#pragma unroll
      for (int k8 = 0; k8 < 32; k8 += 8) {
        T bv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) bv[u] = Xs[32 * h + k8 + u][r16];
        mac8<R>(a + k8, bv, odd, accR, accI);
      }
    } else {
      if constexpr (WAIT)
        chain_wait(fl + J * FLAG_STRIDE, epoch, status);
      else
        __syncthreads();
      chain_fill<R>(Xc + (int64_t)(J * NB) * ldx, ldx, Xs);
      __syncthreads();
#pragma unroll
      for (int k8 = 0; k8 < 32; k8 += 8) {
        T a[8], bv[8];
        load_chunk<R, CONJ>(Ablk, ld, row0, k8, a);
#pragma unroll
        for (int u = 0; u < 8; ++u) bv[u] = Xs[32 * h + k8 + u][r16];
        mac8<R>(a, bv, odd, accR, accI);
      }
    }
  }
}

// Tile position q of chain c (all 256 threads of the workgroup): wait for (or,
// without WAIT, read back) and accumulate the earlier blocks, apply D_I,
// publish x_I.  Every store of x_I has completed when it returns.
template <typename R, bool WAIT>
__device__ __forceinline__ void sweep_tile(int q, int c, int fwd, int nsteps, int cpb, SweepOperand<R> d0,
                                           SweepOperand<R> d1, SweepOperand<R> a0, SweepOperand<R> a1, int split,
                                           cx<R>* X, int64_t sX, int64_t ldx, int* flags, int epoch,
                                           int* status) {
  using T = cx<R>;
  using MF = Mfma<R>;
  using V = typename MF::V;
  constexpr int NB = NB_MAX;
  constexpr bool DS_LDS = sizeof(R) == 4;  // FP32: D_I staged in LDS ahead of use
  __shared__ T Ds[DS_LDS ? NB : 1][NB + 1];
  __shared__ T Rs[NB][17];
  __shared__ T Xs[NB][17];  // x_J of the current dependency; finally x_I
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int bb = c / cpb, c16 = c % cpb;
  const bool second = bb >= split;
  const int hb = second ? bb - split : bb;
  const SweepOperand<R> dop = second ? d1 : d0;
  const SweepOperand<R> aop = second ? a1 : a0;
  const T* W = aop.p + hb * aop.stride;
  T* Xc = X + bb * sX + c16 * 16;
  const int* fl = WAIT ? flags + (int64_t)c * nsteps * FLAG_STRIDE : nullptr;
  const int I = fwd ? q : nsteps - 1 - q;
  const int row0 = 16 * w;
  const T* D = dop.p + hb * dop.stride + (int64_t)I * 2 * NB * NB;

  if constexpr (DS_LDS) {
    for (int e = tid; e < NB * NB; e += 256) {
      const int i = e / NB, k = e % NB;
      Ds[i][k] = dop.conj ? cconj(D[k * NB + i]) : D[i * NB + k];
    }
  }
  // b_I in the product layout: lane (r16, kq), register r holds row MF::row(kq, r)
  T b[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) b[r] = Xc[(int64_t)(I * NB + row0 + MF::row(kq, r)) * ldx + r16];
  V accR = V{0, 0, 0, 0}, accI = V{0, 0, 0, 0};
  if (aop.conj)
    chain_accumulate<R, true, WAIT>(q, I, fwd, nsteps, W, aop.ld, Xc, ldx, row0, fl, epoch, status, Xs, accR, accI);
  else
    chain_accumulate<R, false, WAIT>(q, I, fwd, nsteps, W, aop.ld, Xc, ldx, row0, fl, epoch, status, Xs, accR,
                                     accI);
  // r = b_I - acc, shared by the four waves for the diagonal-block product
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    T v;
    v.x = b[r].x - accR[r];
    v.y = b[r].y - accI[r];
    Rs[row0 + MF::row(kq, r)][r16] = v;
  }
  __syncthreads();
  V xR = V{0, 0, 0, 0}, xI = V{0, 0, 0, 0};
  {
    const int h = kq >> 1;
#pragma unroll
    for (int k8 = 0; k8 < 32; k8 += 8) {
      T a[8], bv[8];
      if constexpr (DS_LDS) {
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = Ds[row0 + r16][32 * h + k8 + u];
      } else if (dop.conj) {
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = cconj(D[(32 * h + k8 + u) * NB + row0 + r16]);
      } else {
        load8(D + (row0 + r16) * NB + 32 * h + k8, a);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) bv[u] = Rs[32 * h + k8 + u][r16];
      mac8<R>(a, bv, kq & 1, xR, xI);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    T v;
    v.x = xR[r];
    v.y = xI[r];
    Xs[row0 + MF::row(kq, r)][r16] = v;  // Xs is free: its last reads preceded the Rs barrier
  }
  __syncthreads();
  chain_publish<R>(Xs, Xc + (int64_t)(I * NB) * ldx, ldx);
  // publish x_I: every wave's stores have completed before the flag is set
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if constexpr (WAIT)
    if (tid == 0) __hip_atomic_store((int*)fl + I * FLAG_STRIDE, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Solution blocks are handed between workgroups without cache maintenance:
// they are written and read with per-access coherent atomics, and a block's
// flag is set only after its stores have completed.
template <typename R>
__global__ __launch_bounds__(256) void k_sweep_chain(int fwd, int nsteps, int nchain, int cpb, SweepOperand<R> d0,
                                                     SweepOperand<R> d1, SweepOperand<R> a0, SweepOperand<R> a1,
                                                     int split, cx<R>* X, int64_t sX, int64_t ldx,
                                                     int* ctl, const int* __restrict__ gate) {
  __shared__ unsigned s_ticket;
  __shared__ int s_epoch, s_run;
  const int tid = threadIdx.x;
  int* status = ctl + SW_STATUS;
  int* flags = ctl + FLAG_STRIDE;
  const unsigned total = (unsigned)(nchain * nsteps);  // == gridDim.x
  if (tid == 0) {
    // the gate is read beside the ticket and the epoch (all three in flight
    // together); a skipped sweep still takes its tickets and re-arms the line
    const unsigned tk = atomicAdd((unsigned*)ctl + SW_TICKET, 1u);
    const int e = __hip_atomic_load(ctl + SW_EPOCH, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int gv = gate != nullptr ? __hip_atomic_load(gate, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 1;
    s_ticket = tk;
    s_epoch = e == INT32_MAX ? 1 : e + 1;
    s_run = gv != 0;
  }
  __syncthreads();
  const unsigned ticket = (unsigned)__builtin_amdgcn_readfirstlane((int)s_ticket);
  const int epoch = __builtin_amdgcn_readfirstlane(s_epoch);
  if (!__builtin_amdgcn_readfirstlane(s_run)) {
    // nothing to solve
  } else if (ticket < total)
    sweep_tile<R, true>((int)(ticket / (unsigned)nchain), (int)(ticket % (unsigned)nchain), fwd, nsteps, cpb, d0, d1,
                        a0, a1, split, X, sX, ldx, flags, epoch, status);
  else if (tid == 0)
    atomicOr(status, 2);
  // the last workgroup to finish re-arms the control line for the next launch
  __syncthreads();
  if (tid == 0 && atomicAdd((unsigned*)ctl + SW_DONE, 1u) == total - 1u) {
    __hip_atomic_store(ctl + SW_TICKET, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(ctl + SW_DONE, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(ctl + SW_EPOCH, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ---------------------------------------------------------------------------
// The same sweep with one workgroup per chain walking all of its tile
// positions in order: no tickets, flags or waits.  The arithmetic of every
// tile is that of k_sweep_chain (same blocks, same order), so both give the
// same bits; this form wins when there are enough chains to fill the device
// (many shifted matrices, short chains), the ticketed one when there are few.
// grid (nchain), block 256.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_sweep_whole(int fwd, int nsteps, int cpb, SweepOperand<R> d0,
                                                     SweepOperand<R> d1, SweepOperand<R> a0, SweepOperand<R> a1,
                                                     int split, cx<R>* X, int64_t sX, int64_t ldx,
                                                     const int* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int c = blockIdx.x;
  for (int q = 0; q < nsteps; ++q)
    sweep_tile<R, false>(q, c, fwd, nsteps, cpb, d0, d1, a0, a1, split, X, sX, ldx, nullptr, 0, nullptr);
}

// After a whole pass: if any one-launch sweep of the plan lost its dependency
// order (the sticky status word of its control line), the status words
// info[0..count) of the plan's problems become `code`.  grid 1, block 64
__global__ void k_sweep_status(const int* __restrict__ ctl, int* __restrict__ info, int count, int code) {
  if (ctl[SW_STATUS] == 0) return;
  for (int i = threadIdx.x; i < count; i += blockDim.x) info[i] = code;
}

// ---------------------------------------------------------------------------
// Row moves of factorization steps [s_begin, s_end) applied to ncols columns:
// forward (P^T, steps in order, new[dst] = old[src]) or inverse (P, steps in
// reverse order, new[src] = old[dst]).  Logical column c is physical column
// c (c < gap_at) or c + gap_len, so the columns on both sides of a panel are
// moved by one launch.  grid (ceil(ncols/CW), batch)
// ---------------------------------------------------------------------------
template <typename R, int CW>
__device__ __forceinline__ void moves_body(int bx, int bb, cx<R>* __restrict__ Bm, int64_t sB, int64_t ldb, int ncols,
                                           int gap_at, int gap_len, const int* __restrict__ moves, int64_t smv,
                                           int s_begin, int s_end, int inverse) {
  using T = cx<R>;
  // each thread holds its (move, column) elements of one step in registers
  // between the reads and the writes: the workgroup's columns are its own, so
  // one barrier orders every read of a step before any of its writes
  constexpr int PER = MOVE_CAP * CW / 256;
  static_assert(MOVE_CAP * CW % 256 == 0, "whole elements per thread");
  Bm += bb * sB;
  const int* mvb = moves + bb * smv;
  const int tid = threadIdx.x;
  const int cb = bx * CW;
  const int ns = s_end - s_begin;
  for (int q = 0; q < ns; ++q) {
    const int step = inverse ? s_end - 1 - q : s_begin + q;
    const int* mv = mvb + (int64_t)step * MOVE_STRIDE;
    const int cnt = mv[0];
    T v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u, i = e / CW, lc = cb + e % CW;
      v[u] = czero<T>();
      if (i < cnt && lc < ncols) {
        const int from = inverse ? mv[1 + i] : mv[1 + MOVE_CAP + i];
        v[u] = Bm[(int64_t)from * ldb + (lc < gap_at ? lc : lc + gap_len)];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + 256 * u, i = e / CW, lc = cb + e % CW;
      if (i < cnt && lc < ncols) {
        const int to = inverse ? mv[1 + MOVE_CAP + i] : mv[1 + i];
        Bm[(int64_t)to * ldb + (lc < gap_at ? lc : lc + gap_len)] = v[u];
      }
    }
    __syncthreads();  // the next step reads what this one wrote
  }
}

template <typename R, int CW>
__global__ __launch_bounds__(256) void k_moves(cx<R>* __restrict__ Bm, int64_t sB, int64_t ldb, int ncols, int gap_at,
                                               int gap_len, const int* __restrict__ moves, int64_t smv, int s_begin,
                                               int s_end, int inverse, const int* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  moves_body<R, CW>(blockIdx.x, blockIdx.y, Bm, sB, ldb, ncols, gap_at, gap_len, moves, smv, s_begin, s_end, inverse);
}

// One factorization step's interchanges on the columns outside its panel
// (workgroups x < gmoves, CW columns each, as k_moves with one step) and the
// inverse of its L11 (the other 4 workgroups per matrix, as k_block_inverse
// with 4 waves and which = 0) in one launch: the two touch disjoint data (the
// moves skip the panel's columns, the inverse reads only the panel's diagonal
// block).  grid (gmoves + 4, batch), block 256
template <typename R, int CW>
__global__ __launch_bounds__(256) void k_moves_inverse(cx<R>* __restrict__ Wb, int64_t wstride, int64_t ld, int ncols,
                                                       int gap_at, int gap_len, const int* __restrict__ moves,
                                                       int64_t smv, int gmoves, int step,
                                                       cx<R>* __restrict__ dinvb, int64_t dstride) {
  __shared__ cx<R> D[NB_MAX][NB_MAX + 1];
  __shared__ cx<R> rdiag[NB_MAX];
  if ((int)blockIdx.x < gmoves)
    moves_body<R, CW>(blockIdx.x, blockIdx.y, Wb, wstride, ld, ncols, gap_at, gap_len, moves, smv, 0, 1, 0);
  else
    block_inverse_body<R, 4>(blockIdx.x - gmoves, blockIdx.y, Wb, wstride, ld, step, 0, dinvb, dstride, D, rdiag);
}

// ---------------------------------------------------------------------------
// Right-hand-side staging: every solution block of the row-major npad x ldS
// array gets its problem's V (column-major n x m, FP64), zero-padded, or the
// identity when V is absent.  Block b (mp columns at b*mp) belongs to pair
// (b mod GP) of the group, i.e. to problem (b mod GP) / P.
// grid-stride over npad*ldS.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_stage(cx<R>* __restrict__ X, int64_t ldS, int npad, int mp, int GP, int P,
                                               const ProblemDesc* __restrict__ descs, ProblemDesc one,
                                               const int* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int64_t total = (int64_t)npad * ldS;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / ldS);
    const int jj = (int)(e % ldS);
    const int b = jj / mp, j = jj % mp;
    const ProblemDesc d = desc_of(descs, one, (b % GP) / P);
    double2 v = czero<double2>();
    if (d.V) {
      if (i < d.n && j < d.m) v = d.V[i + (int64_t)j * d.ldv];
      if (d.real) v.y = 0;
    } else if (i == j && i < d.n) {
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
// theta_p (block g*P+p) and Z_p the one for conj(theta_p) (block GP+g*P+p), in
// FP64 in the fixed pair order (eq. equ:expAx with Remark
// rem:two_time_real_part).  Output column-major n x m of problem g =
// blockIdx.y.  One thread per output element.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_accum_thin(const double2* __restrict__ Xs, int64_t ldS, int mp, int GP, int P,
                                                    const double2* __restrict__ a,
                                                    const ProblemDesc* __restrict__ descs, ProblemDesc one,
                                                    int adjoint_blocks) {
  const int g = blockIdx.y;
  const ProblemDesc d = desc_of(descs, one, g);
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)d.n * d.m) return;
  const int i = (int)(e / d.m), j = (int)(e % d.m);
  const double2* row = Xs + (int64_t)i * ldS;
  double sr = 0, si = 0;
  for (int p = 0; p < P; ++p) {
    double2 ap = a[p];
    ap.x *= d.ec;
    ap.y *= d.ec;
    const double2 y = row[(g * P + p) * mp + j];
    // real data: the conjugate pole's solution is the conjugate of the primal one
    const double2 z = adjoint_blocks ? row[(GP + g * P + p) * mp + j] : cconj(y);
    sr += ap.x * y.x - ap.y * y.y + ap.x * z.x + ap.y * z.y;
    si += ap.x * y.y + ap.y * y.x + ap.x * z.y - ap.y * z.x;
  }
  double2 o;
  o.x = sr;
  o.y = si;
  d.X[i + (int64_t)j * d.ldx] = o;
}

// ---------------------------------------------------------------------------
// K10 (V = I): X = sum_p (a_p Y_p + (a_p Y_p)^H), Y_p = (tA + theta_p I)^{-1}
// (block g*P+p of the solution array, npad columns each): the conjugate
// pole's inverse is the adjoint of Y_p (eq. equ:ExpoMatRat with Remark
// rem:two_time_real_part).  32x32 output tiles through LDS; column-major out.
// grid (ceil(nmax/32), ceil(nmax/32), G), block (32, 8)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_accum_full(const double2* __restrict__ Xs, int64_t ldS, int npad, int P,
                                                    const double2* __restrict__ a,
                                                    const ProblemDesc* __restrict__ descs, ProblemDesc one) {
  __shared__ double2 t1[32][33];
  __shared__ double2 t2[32][33];
  const int g = blockIdx.z;
  const ProblemDesc d = desc_of(descs, one, g);
  const int n = d.n;
  const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;
  if (bi >= n || bj >= n) return;
  const int tx = threadIdx.x, ty = threadIdx.y;
  double sr[4] = {0, 0, 0, 0}, si[4] = {0, 0, 0, 0};
  for (int p = 0; p < P; ++p) {
    const double2* Y = Xs + (int64_t)(g * P + p) * npad;
    __syncthreads();
    for (int q = 0; q < 4; ++q) {
      const int rr = ty + 8 * q;
      t1[rr][tx] = Y[(int64_t)(bi + rr) * ldS + bj + tx];  // (i, j) block
      t2[rr][tx] = Y[(int64_t)(bj + rr) * ldS + bi + tx];  // (j, i) block
    }
    __syncthreads();
    double2 ap = a[p];
    ap.x *= d.ec;
    ap.y *= d.ec;
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
      d.X[i + (int64_t)j * d.ldx] = o;
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

// Largest of the non-negative doubles x and y held by the workgroup's threads, as
// ordered bit patterns (NaN compares above every number), stored to dst[0] and
// dst[1].  Every thread of the (256-thread) workgroup calls it.
__device__ __forceinline__ void block_max2_bits(double x, double y, unsigned long long* dst) {
  __shared__ unsigned long long part[2][4];
  unsigned long long a = (unsigned long long)__double_as_longlong(x);
  unsigned long long b = (unsigned long long)__double_as_longlong(y);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const unsigned long long u = __shfl_xor(a, o), v = __shfl_xor(b, o);
    a = u > a ? u : a;
    b = v > b ? v : b;
  }
  if ((threadIdx.x & 63) == 0) {
    part[0][threadIdx.x >> 6] = a;
    part[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    unsigned long long m = part[threadIdx.x][0];
    for (int w = 1; w < 4; ++w) m = part[threadIdx.x][w] > m ? part[threadIdx.x][w] : m;
    dst[threadIdx.x] = m;
  }
}

// X64 += D32 on solution block b = blockIdx.y (mp columns of the row-major
// npad x ldS arrays).  With `maxima`, also the workgroup's largest correction and
// largest updated entry (max of |Re| and |Im|) into maxima[2w], maxima[2w + 1],
// w = b * gridDim.x + blockIdx.x, for the convergence test.
// grid (any, nblk), block 256: each block's npad*mp elements grid-strided
__global__ __launch_bounds__(256) void k_add_correction(double2* __restrict__ X, const float2* __restrict__ D,
                                                        int64_t ldS, int npad, int mp,
                                                        unsigned long long* __restrict__ maxima,
                                                        const int* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int blk = blockIdx.y;
  double dm = 0.0, xm = 0.0;
  const int64_t count = (int64_t)npad * mp;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = (q / mp) * ldS + (int64_t)blk * mp + q % mp;
    const float2 d = D[e];
    double2 x = X[e];
    x.x += (double)d.x;
    x.y += (double)d.y;
    X[e] = x;
    // (fmax would drop a NaN: the comparison form keeps it)
    const double a = fabs((double)d.x), b = fabs((double)d.y);
    const double m1 = !(a <= b) ? a : b;
    dm = !(m1 <= dm) ? m1 : dm;
    xm = fmax(xm, fmax(fabs(x.x), fabs(x.y)));
  }
  if (maxima != nullptr)
    block_max2_bits(dm, xm, maxima + 2 * ((int64_t)blk * gridDim.x + blockIdx.x));
}

// Start of the refinement sweeps: gate open, the check's finish counter cleared,
// every problem's flag set to `nc0`.  grid 1, block 256
__global__ __launch_bounds__(256) void k_ir_begin(int* __restrict__ gate, int* __restrict__ ir_nc, int G, int nc0,
                                                  unsigned* __restrict__ done) {
  for (int g = threadIdx.x; g < G; g += blockDim.x) ir_nc[g] = nc0;
  if (threadIdx.x == 0) {
    *gate = 1;
    *done = 0u;
  }
}

// Refinement right-hand side in FP32 on solution block b = blockIdx.y:
//   out = Rres - sum_{s < nparts} part[s*pstride + e] - shift_b * X
// Rres holds the staged V (minus the product, when nparts = 0); part the split-K
// partial products of (t A) X, summed in slice order.  Block b's shift: primal
// blocks (b < GP) theta - c of pair b mod P (c the problem's shift), adjoint
// blocks its conjugate.
// grid (any, nblk), block 256: each block's npad*mp elements grid-strided
__global__ __launch_bounds__(256) void k_residual32(const double2* __restrict__ Rres, const double2* __restrict__ part,
                                                    int nparts, int64_t pstride, const double2* __restrict__ X,
                                                    int64_t ldS, int npad, int mp, int GP, int P,
                                                    const double2* __restrict__ theta,
                                                    const ProblemDesc* __restrict__ descs, ProblemDesc one,
                                                    float2* __restrict__ out, const int* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int blk = blockIdx.y;
  double2 th = theta[(blk % GP) % P];
  th.x -= desc_of(descs, one, (blk % GP) / P).c;
  if (blk >= GP) th.y = -th.y;
  const int64_t count = (int64_t)npad * mp;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = (q / mp) * ldS + (int64_t)blk * mp + q % mp;
    double2 sum = {0.0, 0.0};
    for (int s = 0; s < nparts; ++s) {
      const double2 p = part[s * pstride + e];
      sum.x += p.x;
      sum.y += p.y;
    }
    const double2 x = X[e];
    double2 r = Rres[e];
    r.x -= sum.x;
    r.y -= sum.y;
    r.x -= th.x * x.x - th.y * x.y;
    r.y -= th.x * x.y + th.y * x.x;
    float2 o;
    o.x = (float)r.x;
    o.y = (float)r.y;
    out[e] = o;
  }
}

// After a refinement sweep (the per-workgroup maxima of k_add_correction, wpb
// workgroups per block): block b has converged when its largest correction is
// at most tol times its largest solution entry (a NaN never converges).  One
// workgroup per block writes conv[b]; the last one to finish (counted in *done)
// sets ir_nc[g] = 1 for each problem g with a block that has not converged (0
// otherwise) and *gate = 1 while any block has not (the next sweep runs), 0
// once all have (its kernels return at once), and clears *done.
// Blocks: primal b = g*P + p (b < GP), adjoint GP + g*P + p when present.
// grid (nblk), block 64
__global__ __launch_bounds__(64) void k_ir_check(const unsigned long long* __restrict__ maxima, int nblk, int wpb,
                                                 int GP, int P, double tol, int* __restrict__ gate,
                                                 int* __restrict__ ir_nc, int* __restrict__ conv,
                                                 unsigned* __restrict__ done) {
  const int b = blockIdx.x, lane = threadIdx.x;
  unsigned long long dmb = 0ull, xmb = 0ull;
  for (int w = lane; w < wpb; w += 64) {
    const unsigned long long u = maxima[2 * ((int64_t)b * wpb + w)];
    const unsigned long long v = maxima[2 * ((int64_t)b * wpb + w) + 1];
    dmb = u > dmb ? u : dmb;
    xmb = v > xmb ? v : xmb;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const unsigned long long u = __shfl_xor(dmb, o), v = __shfl_xor(xmb, o);
    dmb = u > dmb ? u : dmb;
    xmb = v > xmb ? v : xmb;
  }
  __shared__ bool last;
  if (lane == 0) {
    const double dm = __longlong_as_double((long long)dmb), xm = __longlong_as_double((long long)xmb);
    conv[b] = dm <= tol * xm ? 1 : 0;
    __threadfence();
    last = atomicAdd(done, 1u) == (unsigned)nblk - 1u;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  const int G = GP / P;
  int any = 0;
  for (int g = lane; g < G; g += 64) {
    int nc = 0;
    for (int b0 = g * P; b0 < nblk; b0 += GP)
      for (int p = 0; p < P; ++p) nc |= __hip_atomic_load(conv + b0 + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    ir_nc[g] = nc;
    any |= nc;
  }
  any = __any(any);
  if (lane == 0) {
    *gate = any ? 1 : 0;
    *done = 0u;
  }
}

// ---------------------------------------------------------------------------
// Refinement residual with double-double accumulation (two FP64 words, error-
// free products by FMA and error-free sums):
//   out = fl32( V - (t A) X - shift_b X )
// for every 16-column group of the npad x ldS right-hand-side array.  V is the
// staged right-hand side (Rv), Ah the FP64 t*A of the group's problem
// (row-major, problem g at Ah + g*nn), shift as in k_residual32.  The error of
// the accumulated sum is of order u^2 * sum |terms| instead of u * sum |terms|,
// so refinement converges past the FP64 residual's limit when the shifted
// matrices are ill conditioned.
// grid (npad/64, ldS/16), block 256: thread (tx, ty) = (tid % 16, tid / 16)
// owns rows r0 + ty + 16a (a = 0..3) of column c0 + tx.
// ---------------------------------------------------------------------------
struct DD {
  double hi, lo;
};
// s += a*b exactly up to the final rounding of (hi, lo)
__device__ __forceinline__ void dd_fma(DD& s, double a, double b) {
  const double p = a * b;
  const double e = fma(a, b, -p);
  const double t = s.hi + p;
  const double bp = t - s.hi;
  const double err = (s.hi - (t - bp)) + (p - bp);
  s.hi = t;
  s.lo += err + e;
}

__global__ __launch_bounds__(256) void k_residual_dd(const double2* __restrict__ Ah, int64_t nn,
                                                     const double2* __restrict__ X, const double2* __restrict__ Rv,
                                                     int64_t ldS, int npad, int mp, int GP, int P,
                                                     const double2* __restrict__ theta,
                                                     const ProblemDesc* __restrict__ descs, ProblemDesc one,
                                                     float2* __restrict__ out, const int* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  constexpr int KC = 16;
  __shared__ double2 As[64][KC + 1];
  __shared__ double2 Xs[KC][16];
  const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
  const int r0 = blockIdx.x * 64;
  const int64_t c0 = (int64_t)blockIdx.y * 16;
  const int blk = (int)(c0 / mp);
  const int g = (blk % GP) / P;
  const double2* A = Ah + (int64_t)g * nn;
  DD re[4], im[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) re[a] = im[a] = DD{0.0, 0.0};
  for (int k0 = 0; k0 < npad; k0 += KC) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q, i = e / KC, k = e % KC;
      As[i][k] = A[(int64_t)(r0 + i) * npad + k0 + k];
    }
    Xs[ty][tx] = X[(int64_t)(k0 + ty) * ldS + c0 + tx];
    __syncthreads();
#pragma unroll 4
    for (int k = 0; k < KC; ++k) {
      const double2 x = Xs[k][tx];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const double2 av = As[ty + 16 * a][k];
        dd_fma(re[a], av.x, x.x);
        dd_fma(re[a], -av.y, x.y);
        dd_fma(im[a], av.x, x.y);
        dd_fma(im[a], av.y, x.x);
      }
    }
    __syncthreads();
  }
  double2 th = theta[(blk % GP) % P];
  th.x -= desc_of(descs, one, g).c;
  if (blk >= GP) th.y = -th.y;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    const int64_t e = (int64_t)(r0 + ty + 16 * a) * ldS + c0 + tx;
    const double2 x = X[e];
    dd_fma(re[a], th.x, x.x);
    dd_fma(re[a], -th.y, x.y);
    dd_fma(im[a], th.x, x.y);
    dd_fma(im[a], th.y, x.x);
    const double2 v = Rv[e];
    float2 o;
    o.x = (float)((v.x - re[a].hi) - re[a].lo);
    o.y = (float)((v.y - im[a].hi) - im[a].lo);
    out[e] = o;
  }
}

}  // namespace
}  // namespace expm

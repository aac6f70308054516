// Shared by the banded and tridiagonal routes: the one-wave banded elimination
// chain (band matrices with kd <= 3, rows given row-major inside the band) and
// its helpers.  Included by one translation unit each; everything is internal.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"

namespace {

using namespace expm;

// pivot magnitude |Re| + |Im|; NaN ranks highest so that it reaches the result
__device__ __forceinline__ double pivot_mag(double2 z) {
  const double m = fabs(z.x) + fabs(z.y);
  return m != m ? INFINITY : m;
}

// LDS-only wait and workgroup barrier: global loads (the next block's inputs) and
// stores (the previous block's outputs) stay in flight across it
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt and expcnt left at their maxima
  __builtin_amdgcn_s_barrier();
}

// ---- narrow bands: one wave per (pole, block of 16 right-hand sides) -----------
// The chain touches only registers and LDS.  Every NB_B columns the wave moves
// the next block's inputs (rows of R and of V, loaded a whole block earlier) into
// LDS, writes the previous block's outputs (rows of U and Y) back, and issues the
// loads of the block after; so every wait on memory covers operations issued a
// block earlier.
// U: row j at U + (k*chunks + chunk)*ustride + j*(2KD+1): [1/pivot, U(j, j+1), ...,
// U(j, j+2KD)] (each block of right-hand sides keeps its own copy)
// Y: pole k's n x m solution, row-major (element (j, r) at Y + k*ystride + j*m + r)
constexpr int NB_B = 32;   // columns per block
constexpr int NB_MC = 16;  // right-hand sides per wave
// R and Vr may hold one matrix and one V per pole (rstride, vstride > 0) or one
// for all poles (0).
template <int KD>
__global__ __launch_bounds__(64) void k_band_narrow(int n, int m, const double2* __restrict__ R,
                                                    const double2* __restrict__ Vr, const double2* __restrict__ pole,
                                                    double2* __restrict__ U, double2* __restrict__ Y,
                                                    int64_t ustride, int64_t ystride, int64_t rstride,
                                                    int64_t vstride) {
  constexpr int W = 2 * KD + 1, B = NB_B, MC = NB_MC;
  constexpr int RCH = (B * W + 63) / 64;  // 64-value pieces of a block of R (or U) rows
  constexpr int VCH = B * MC / 64;        // ... of a block of V (or Y) rows
  __shared__ double2 sR[B * W], sV[B * MC], sU[B * W], sY[B * MC];
  const int k = blockIdx.x, lane = threadIdx.x;
  const int rc = blockIdx.y * MC, r = rc + lane;
  const bool act = lane < MC && r < m;
  const double2 th = pole[k];
  double2* Uk = U + ((int64_t)k * gridDim.y + blockIdx.y) * ustride;
  double2* Yk = Y + k * ystride;
  R += k * rstride;
  Vr += k * vstride;
  const int nblk = (n + B - 1) / B;
  double2 gR[RCH], gV[VCH];
  // rows q0 .. q0+B-1 of R and of this wave's columns of a row-major n x m array
  auto load_rows = [&](const double2* src, int64_t q0, int64_t ld_src) {
#pragma unroll
    for (int c = 0; c < RCH; ++c) {
      const int f = c * 64 + lane;
      const int64_t e = q0 * W + f;
      gR[c] = (f < B * W && q0 + f / W < n) ? src[e] : czero<double2>();
    }
    (void)ld_src;
  };
  auto load_cols = [&](const double2* src, int64_t q0) {
#pragma unroll
    for (int c = 0; c < VCH; ++c) {
      const int f = c * 64 + lane, i = f / MC, cc = f % MC;
      const int64_t q = q0 + i;
      gV[c] = (q < n && rc + cc < m) ? src[q * m + rc + cc] : czero<double2>();
    }
  };
  auto stage = [&](double2* dR, double2* dV) {
#pragma unroll
    for (int c = 0; c < RCH; ++c)
      if (c * 64 + lane < B * W) dR[c * 64 + lane] = gR[c];
#pragma unroll
    for (int c = 0; c < VCH; ++c) dV[c * 64 + lane] = gV[c];
  };
  // rows j0 .. j0+rows-1 of U (from sU, if given) and of this wave's columns of Y
  auto flush = [&](const double2* srcU, const double2* srcY, int j0, int rows) {
    if (srcU) {
#pragma unroll
      for (int c = 0; c < RCH; ++c) {
        const int f = c * 64 + lane;
        if (f < rows * W) Uk[(int64_t)j0 * W + f] = srcU[f];
      }
    }
#pragma unroll
    for (int c = 0; c < VCH; ++c) {
      const int f = c * 64 + lane, i = f / MC, cc = f % MC;
      if (i < rows && rc + cc < m) Yk[(int64_t)(j0 + i) * m + rc + cc] = srcY[f];
    }
  };

  // ---- forward: elimination with partial pivoting, V transformed alongside ----
  double2 w[KD + 1][W], bb[KD + 1];
#pragma unroll
  for (int i = 0; i <= KD; ++i) {
#pragma unroll
    for (int c = 0; c < W; ++c) {
      const int off = c - i + KD;  // column c of row i
      double2 v = czero<double2>();
      if (i < n && off >= 0 && off < W) {
        v = R[(int64_t)i * W + off];
        if (c == i) {
          v.x += th.x;
          v.y += th.y;
        }
      }
      w[i][c] = v;
    }
    bb[i] = (act && i < n) ? Vr[(int64_t)i * m + r] : czero<double2>();
  }
  // block b inserts rows b*B + KD + 1 .. b*B + KD + B
  load_rows(R, KD + 1, 0);
  load_cols(Vr, KD + 1);
  for (int b = 0; b < nblk; ++b) {
    const int j0 = b * B;
    stage(sR, sV);
    if (b > 0) flush(sU, sY, j0 - B, B);
    if (b + 1 < nblk) {
      load_rows(R, (int64_t)j0 + B + KD + 1, 0);
      load_cols(Vr, (int64_t)j0 + B + KD + 1);
    }
    const int jn = min(B, n - j0);
    for (int jj = 0; jj < jn; ++jj) {
      const int j = j0 + jj;
      const bool qin = j + KD + 1 < n;
      // the row inserted at the end of this step (read now, used last)
      double2 nr[W];
#pragma unroll
      for (int c = 0; c < W; ++c) nr[c] = sR[jj * W + c];
      const double2 nb = sV[jj * MC + (lane & (MC - 1))];
      const int alive = min(KD + 1, n - j);  // window rows that hold matrix rows
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
      const double2 rp = crecip_fast(w[0][0]);
#pragma unroll
      for (int i = 1; i <= KD; ++i) {
        const double2 l = cmul(w[i][0], rp);
#pragma unroll
        for (int c = 1; c < W; ++c) w[i][c] = cfms(w[i][c], l, w[0][c]);
        bb[i] = cfms(bb[i], l, bb[0]);
      }
      if (lane < W) {  // row j of U: lane c writes entry c
        double2 u = rp;
#pragma unroll
        for (int c = 1; c < W; ++c)
          if (lane == c) u = w[0][c];
        sU[jj * W + lane] = u;
      }
      if (lane < MC) sY[jj * MC + lane] = bb[0];
      // the window moves one row down and one column right; the new row is matrix
      // row j + KD + 1 over columns j + 1 .. j + 1 + 2KD (row jj of the block's R)
#pragma unroll
      for (int i = 0; i < KD; ++i) {
#pragma unroll
        for (int c = 0; c + 1 < W; ++c) w[i][c] = w[i + 1][c + 1];
        w[i][W - 1] = czero<double2>();
        bb[i] = bb[i + 1];
      }
#pragma unroll
      for (int c = 0; c < W; ++c) {
        double2 v = qin ? nr[c] : czero<double2>();
        if (c == KD && qin) {
          v.x += th.x;
          v.y += th.y;
        }
        w[KD][c] = v;
      }
      bb[KD] = (qin && lane < MC) ? nb : czero<double2>();
    }
  }
  flush(sU, sY, (nblk - 1) * B, n - (nblk - 1) * B);
  __syncthreads();  // the rows written above are read back below (other lanes)

  // ---- back substitution, blocks from the last to the first --------------------
  // x_j = (1/u_jj)(y_j - sum_c u_{j,j+c} x_{j+c}), in place in Y
  double2 xs[2 * KD + 1];  // xs[c - 1] = x_{j + c}
#pragma unroll
  for (int c = 0; c < 2 * KD + 1; ++c) xs[c] = czero<double2>();
  load_rows(Uk, (int64_t)(nblk - 1) * B, 0);
  load_cols(Yk, (int64_t)(nblk - 1) * B);
  for (int b = nblk - 1; b >= 0; --b) {
    const int j0 = b * B;
    stage(sR, sV);  // U rows and y of block b
    if (b + 1 < nblk) flush(nullptr, sY, j0 + B, min(B, n - j0 - B));
    if (b > 0) {
      load_rows(Uk, (int64_t)j0 - B, 0);
      load_cols(Yk, (int64_t)j0 - B);
    }
    const int jn = min(B, n - j0);
    // each step's row of U and y are read one step ahead
    double2 un[W], yn;
#pragma unroll
    for (int c = 0; c < W; ++c) un[c] = sR[(jn - 1) * W + c];
    yn = sV[(jn - 1) * MC + (lane & (MC - 1))];
    for (int jj = jn - 1; jj >= 0; --jj) {
      double2 u[W];
#pragma unroll
      for (int c = 0; c < W; ++c) u[c] = un[c];
      double2 s = lane < MC ? yn : czero<double2>();
      if (jj > 0) {
#pragma unroll
        for (int c = 0; c < W; ++c) un[c] = sR[(jj - 1) * W + c];
        yn = sV[(jj - 1) * MC + (lane & (MC - 1))];
      }
#pragma unroll
      for (int c = 1; c < W; ++c) s = cfms(s, u[c], xs[c - 1]);
      const double2 x = cmul(u[0], s);
#pragma unroll
      for (int c = 2 * KD; c >= 1; --c) xs[c] = xs[c - 1];
      xs[0] = x;
      if (lane < MC) sY[jj * MC + lane] = x;
    }
  }
  flush(nullptr, sY, 0, min(B, n));
}

}  // namespace

// Device-side building blocks shared by the kernels of libexpm_pfd (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace expm {

// Interleaved complex element type for each real type.
template <typename R>
struct CxT;
template <>
struct CxT<double> {
  using T = double2;
};
template <>
struct CxT<float> {
  using T = float2;
};
template <typename R>
using cx = typename CxT<R>::T;

template <typename T>
__device__ __forceinline__ T czero() {
  T z;
  z.x = 0;
  z.y = 0;
  return z;
}
template <typename T>
__device__ __forceinline__ T cmul(T a, T b) {
  T r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
// c - a*b
template <typename T>
__device__ __forceinline__ T cfms(T c, T a, T b) {
  T r;
  r.x = c.x - a.x * b.x + a.y * b.y;
  r.y = c.y - a.x * b.y - a.y * b.x;
  return r;
}
template <typename T>
__device__ __forceinline__ T cconj(T a) {
  a.y = -a.y;
  return a;
}
// 1/a with the larger component scaled out (Smith-style), so |a| far from 1 stays accurate
template <typename T>
__device__ __forceinline__ T crecip(T a) {
  T r;
  if (fabs(a.x) >= fabs(a.y)) {
    auto q = a.y / a.x;
    auto den = a.x + a.y * q;
    r.x = 1 / den;
    r.y = -q / den;
  } else {
    auto q = a.x / a.y;
    auto den = a.x * q + a.y;
    r.x = q / den;
    r.y = -1 / den;
  }
  return r;
}
// reciprocal from the hardware estimate refined by Newton steps (one in FP32,
// two in FP64: the FP64 estimate is good to about 2^-22)
__device__ __forceinline__ float rcp_nr(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
// 1/a by the same scaling as crecip, with reciprocals instead of divisions
template <typename T>
__device__ __forceinline__ T crecip_fast(T a) {
  const bool re_big = fabs(a.x) >= fabs(a.y);
  const auto big = re_big ? a.x : a.y, small = re_big ? a.y : a.x;
  const auto q = small * rcp_nr(big);
  const auto rd = rcp_nr(big + small * q);
  T r;
  r.x = re_big ? rd : q * rd;
  r.y = re_big ? -q * rd : -rd;
  return r;
}

template <typename T>
__device__ __forceinline__ T cdiv(T a, T b) {
  return cmul(a, crecip(b));
}

// ---- matrix-core products -------------------------------------------------
// One 16x16x4 real product per call.  Operand layout (checked on gfx950):
//   A[i][k] comes from lane i + 16k, B[k][j] from lane j + 16k.
// Result layout differs between the two types:
//   f64: lane l, register r holds D[l/16 + 4r][l%16]
//   f32: lane l, register r holds D[4(l/16) + r][l%16]
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename R>
struct Mfma;
template <>
struct Mfma<double> {
  using V = d4;
  static __device__ __forceinline__ V run(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kq, int r) { return kq + 4 * r; }
};
template <>
struct Mfma<float> {
  using V = f4;
  static __device__ __forceinline__ V run(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int kq, int r) { return 4 * kq + r; }
};

// ---- wave-wide reductions through DPP (gfx9 row broadcasts) ---------------
// dpp_ctrl codes: quad_perm [1,0,3,2] = 0xB1, [2,3,0,1] = 0x4E, row_half_mirror
// = 0x141, row_mirror = 0x140, row_bcast:15 = 0x142, row_bcast:31 = 0x143.
// Lanes whose DPP source is masked off keep their own value (old = src).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(v, v, CTRL, ROWMASK, 0xF, false);
}
// max (min) of v and the DPP-moved v.  The identity of the operation as the
// value of lanes whose source is masked off lets the compiler fold the move
// into the max (min) instruction itself; such lanes keep v.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_max_i32(int v) {
  return max(v, __builtin_amdgcn_update_dpp((int)0x80000000, v, CTRL, ROWMASK, 0xF, false));
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_min_i32(int v) {
  return min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, CTRL, ROWMASK, 0xF, false));
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(dpp_i32<CTRL, ROWMASK>(__float_as_int(v)));
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i32<CTRL, ROWMASK>((int)(b & 0xffffffffll));
  const int hi = dpp_i32<CTRL, ROWMASK>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// maximum over the 16 lanes of each row, valid in every lane of the row
template <typename R>
__device__ __forceinline__ R row16_max(R x) {
  x = fmax(x, dpp_move<0xB1, 0xF>(x));
  x = fmax(x, dpp_move<0x4E, 0xF>(x));
  x = fmax(x, dpp_move<0x141, 0xF>(x));
  x = fmax(x, dpp_move<0x140, 0xF>(x));
  return x;
}
__device__ __forceinline__ int row16_min(int x) {
  x = dpp_min_i32<0xB1, 0xF>(x);
  x = dpp_min_i32<0x4E, 0xF>(x);
  x = dpp_min_i32<0x141, 0xF>(x);
  x = dpp_min_i32<0x140, 0xF>(x);
  return x;
}
// maximum over the wave, returned in every lane
template <typename R>
__device__ __forceinline__ R wave_max(R x) {
  x = row16_max(x);
  x = fmax(x, dpp_move<0x142, 0xA>(x));
  x = fmax(x, dpp_move<0x143, 0xC>(x));
  if constexpr (sizeof(R) == 8) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  } else {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
  }
}
__device__ __forceinline__ int wave_min(int x) {
  x = row16_min(x);
  x = dpp_min_i32<0x142, 0xA>(x);
  x = dpp_min_i32<0x143, 0xC>(x);
  return __builtin_amdgcn_readlane(x, 63);
}

// Value of lane k (k uniform across the wave) in every lane.
__device__ __forceinline__ float lane_bcast(float v, int k) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ __forceinline__ double lane_bcast(double v, int k) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), k);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename T>
__device__ __forceinline__ T lane_bcast2(T v, int k) {
  T r;
  r.x = lane_bcast(v.x, k);
  r.y = lane_bcast(v.y, k);
  return r;
}

// ---- device-coherent 16-byte accesses ------------------------------------------
// Raw buffer resource over [p, p + bytes): loads past the end return zero and
// stores past it are dropped.  Accesses with the SC1 cache policy are coherent
// across the device's CUs and XCDs without cache-wide maintenance (the same
// policy the compiler gives relaxed agent-scope atomics).
typedef unsigned int u32x4 __attribute__((__vector_size__(4 * sizeof(unsigned int))));
constexpr int CPOL_SC1 = 16;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ u32x4 coherent_load16(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, CPOL_SC1);
}
__device__ __forceinline__ void coherent_store16(u32x4 v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)off, 0, CPOL_SC1);
}

// ---- problem descriptors ----------------------------------------------------
// One exp(t A) V problem as the caller laid it out (column-major, FP64 complex).
struct ProblemDesc {
  const double2* A;
  int64_t lda;
  const double2* V;  // nullptr: V = I
  int64_t ldv;
  double2* X;
  int64_t ldx;
  double t;
  int n, m;
  int real;   // 1: A and V are real; their imaginary parts are not read
  int upper;  // 1: the upper triangle of A is read instead of the lower one
  int* info;  // device word for this problem's status (0, 1: refinement missed its
              // tolerance, 2: non-finite result); may be null
  double c;   // shift of the shifting method in units of tA (0: none): the problem's
              // poles are theta_k - c and its residues e^c a_k
  double ec;  // e^c, rounded once on the host
};
// descriptor g of a group: from the device array, or the single inline one
__device__ __forceinline__ ProblemDesc desc_of(const ProblemDesc* arr, const ProblemDesc& one, int g) {
  return arr ? arr[g] : one;
}

// ---- row interchanges -----------------------------------------------------
// Row moves of one factorization step are stored as
//   [count, dst[0..MOVE_CAP), src[0..MOVE_CAP)]
// meaning: after the step's interchanges, row dst[e] holds what row src[e] held.
constexpr int NB_MAX = 64;                 // widest outer panel
constexpr int MOVE_CAP = 2 * NB_MAX;       // at most 2 moves per interchange
constexpr int MOVE_STRIDE = 1 + 2 * MOVE_CAP;

// Run by one full wave.  Simulates the interchanges (base+i) <-> piv[i],
// i = 0..cnt-1 (cnt <= 64, piv[i] >= base+i, applied in order), and writes the
// net row moves to dst/src.  Returns the number of moves (same on all lanes).
// piv is read once (one element per lane); every later exchange of values
// between lanes uses readlane with a wave-uniform lane index.  If slot_of is
// given, slot_of[i] (i < cnt) is the index of the move that fills row base+i,
// or -1 if that row keeps its value.
__device__ inline int composite_moves(const int* piv, int cnt, int base, int* dst, int* src,
                                      int* slot_of = nullptr) {
  const int lane = threadIdx.x & 63;
  const int mypiv = lane < cnt ? piv[lane] : 0;
  int cur = base + lane;  // original row now at position base+lane
  int key = -1, val = 0;  // one position outside [base, base+cnt) tracked by this lane
  for (int i = 0; i < cnt; ++i) {
    const int b = __builtin_amdgcn_readlane(mypiv, i);
    const int ta = __builtin_amdgcn_readlane(cur, i);
    if (b < base + cnt) {
      const int tb = __builtin_amdgcn_readlane(cur, b - base);
      if (lane == i) cur = tb;
      if (lane == b - base) cur = ta;
    } else {
      const unsigned long long m = __ballot(key == b);
      int slot, tb;
      if (m) {
        slot = __ffsll((long long)m) - 1;
        tb = __builtin_amdgcn_readlane(val, slot);
      } else {
        slot = i;
        tb = b;
      }
      if (lane == i) cur = tb;
      if (lane == slot) {
        key = b;
        val = ta;
      }
    }
  }
  const bool pt = lane < cnt && cur != base + lane;
  const bool po = key >= 0 && val != key;
  const unsigned long long mt = __ballot(pt), mo = __ballot(po);
  const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  const int nt = __popcll(mt);
  if (pt) {
    const int pos = __popcll(mt & below);
    dst[pos] = base + lane;
    src[pos] = cur;
  }
  if (po) {
    const int pos = nt + __popcll(mo & below);
    dst[pos] = key;
    src[pos] = val;
  }
  if (slot_of != nullptr && lane < cnt) slot_of[lane] = pt ? __popcll(mt & below) : -1;
  return nt + __popcll(mo);
}

}  // namespace expm

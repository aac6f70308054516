// Host-side argument checks shared by the library's translation units.
#pragma once

#include <cmath>
#include <cstdint>

#include "../../include/expm_pfd.h"
#include "device_common.h"

namespace expm {

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// number of LU trailing-update tile shapes (option lu_tile takes 0..LU_TILE_COUNT)
constexpr int LU_TILE_COUNT = 3;

inline int check_degree(int degree) {
  return (degree < 2 || degree > EXPM_PFD_MAX_DEGREE || (degree & 1)) ? EXPM_PFD_ERR_DEGREE : 0;
}

inline int check_opts(const expm_pfd_opts* o) {
  if (!o) return 0;
  if (o->precision != EXPM_PFD_FP64 && o->precision != EXPM_PFD_MIXED) return EXPM_PFD_ERR_ARG;
  if (o->lu_tile < 0 || o->lu_tile > LU_TILE_COUNT) return EXPM_PFD_ERR_ARG;
  if (o->uplo != EXPM_PFD_LOWER && o->uplo != EXPM_PFD_UPPER) return EXPM_PFD_ERR_ARG;
  if (!std::isfinite(o->shift)) return EXPM_PFD_ERR_ARG;
  if (!o->shift_scale_t && !std::isfinite(std::exp(o->shift))) return EXPM_PFD_ERR_ARG;
  if (std::isnan(o->ir_tol)) return EXPM_PFD_ERR_ARG;
  if (o->tridiag_reuse < 0) return EXPM_PFD_ERR_ARG;
  return 0;
}

// Shift of one problem in units of its tA (c = shift, or t * shift when the
// shift is given in units of A) and e^c; EXPM_PFD_ERR_ARG if e^c overflows.
inline int problem_shift(double shift, int scale_t, double t, ProblemDesc& d) {
  d.c = scale_t ? t * shift : shift;
  d.ec = std::exp(d.c);
  return std::isfinite(d.c) && std::isfinite(d.ec) ? 0 : EXPM_PFD_ERR_ARG;
}

// Tridiagonal-route plans with their device memory from the stream-ordered
// pool on `pool` (the serving queue's use; nullptr: hipMalloc), and their
// release on a stream (the plan's work must be complete or ordered before it).
// Defined with the route (tridiag.hip).
int tri_create(expm_pfd_tri_t* out, int64_t n, int degree, int64_t m_max, const expm_pfd_opts* opts,
               hipStream_t pool);
void tri_release(expm_pfd_tri_t tri, hipStream_t stream);
// device bytes tri_create allocates
size_t tri_bytes(int64_t n, int degree, int64_t m_max);

}  // namespace expm

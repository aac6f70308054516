// libexpm_pfd: exp(tA)V ~ R_d(tA)V for Hermitian A on gfx950 (see include/expm_pfd.h).
//
// apply(), FP64 path:
//   K1 form W_p = tA + theta_p I for the d/2 pole pairs (one launch, all pairs)
//   LU with partial pivoting of every W_p (right-looking, outer panels of 64
//     columns split into register-resident inner panels; every launch covers
//     all pairs):
//       per inner panel: K2 panel factorization, K5 update of the rest of the
//       outer panel;  per outer panel: row moves on the left columns,
//       K4 interchanges + triangular solve for the U12 block row, K5 trailing
//       update A22 -= L21 U12 on the matrix cores.
//   solves: Y_p = W_p^{-1} V (primal) and Z_p = (W_p^H)^{-1} V (conjugate pole,
//     same factors: W_p^H = U^H L^H P^T), right-looking block sweeps
//     (K4 diagonal block + K5 update), all pairs per launch.
//   K10 X = sum_p a_p Y_p + conj(a_p) Z_p in FP64 (for V = I: Y_p + Y_p^H form).
// MIXED path: the same factorization and solves in complex FP32, then per
//   sweep an FP64 residual R = V - (tA + theta I) X for all pole solves as one
//   matrix-core product with the shared FP64 tA, a FP32 correction solve and an
//   FP64 update; accumulation in FP64.

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "../../include/expm_pfd.h"
#include "host_common.h"
#include "kernels.h"

using namespace expm;

namespace {

constexpr int NB = 64;  // outer panel width (also the padding granularity)
constexpr int CHAIN_MP_MAX = 64;  // widest right-hand-side block solved by one-launch sweeps
// from this many 16-column chains on, a sweep runs one workgroup per chain
// (k_sweep_whole) instead of one per tile position (k_sweep_chain)
constexpr int WHOLE_CHAIN_MIN = 256;

// ---- per-launch event tracing (expm_pfd_trace) ---------------------------------
namespace trace {
struct Rec {
  hipEvent_t a, b;
  int cls;
  double flops, bytes;
};
unsigned mask = 0;  // bit c set: launches of kernel class c are timed
std::vector<Rec> recs;
std::mutex mu;  // records may come from the serving thread
std::vector<hipEvent_t> pool;
hipEvent_t get_event() {
  std::lock_guard<std::mutex> lk(mu);
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}
void clear() {
  for (auto& r : recs) {
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.clear();
}
// Brackets one kernel launch with an event pair on its stream.  With `in_launch`
// the pair is handed to the launch itself (hipExtLaunchKernelGGL records it at the
// kernel's own start and end), so the time excludes the separate event packets.
struct Scope {
  bool active, in_launch;
  hipStream_t s;
  Rec r{};
  Scope(hipStream_t st, int cls, double flops, double bytes, bool in_launch_ = false)
      : active((mask >> cls) & 1u), in_launch(in_launch_), s(st) {
    if (active) {
      r = {get_event(), get_event(), cls, flops, bytes};
      if (!in_launch) (void)hipEventRecord(r.a, s);
    }
  }
  ~Scope() {
    if (active) {
      if (!in_launch) (void)hipEventRecord(r.b, s);
      std::lock_guard<std::mutex> lk(mu);
      recs.push_back(r);
    }
  }
};
}  // namespace trace

struct HipErr {
  hipError_t e = hipSuccess;
  void operator()(hipError_t x) {
    if (x != hipSuccess && e == hipSuccess) e = x;
  }
};

// Inner panel width: the register panel holds IB columns of ceil(npad/PANEL_NT)
// rows per thread (<= 32 complex per thread in FP64, 64 in FP32: 128 registers)
// and is staged through a PANEL_NT x IB LDS buffer of 64 KB.
int inner_width(int64_t npad, bool fp64) {
  if (fp64) return npad <= 2048 ? 8 : npad <= 4096 ? 4 : 2;
  return npad <= 2048 ? 16 : npad <= 4096 ? 8 : 4;
}
// inner width of the panels of one outer step: FP64 panels of at most 1024 rows
// take 16 columns (two rows per thread), the others the plan's width
int inner_width_at(int ib, int rows, bool fp64) { return fp64 && ib == 8 && rows <= 1024 ? 16 : ib; }

// ---- launch helpers ---------------------------------------------------------

struct PanelArgs {
  int64_t ws, ld, ps, ms;
  int P, npad, j0, c0, nbo, step, last;
  int* ipiv;
  int* moves;
};

template <typename R, int IB, int S>
void panel_launch(hipStream_t st, const PanelArgs& g, cx<R>* W) {
  const int P = g.P;
  constexpr int LIMIT = sizeof(R) == 8 ? 32 : 64;
  // widths inner_width and inner_width_at can choose: FP32 16/8/4, FP64 16/8/4/2
  if constexpr (IB * S <= LIMIT && (sizeof(R) == 4 ? IB >= 4 && IB <= 16 : IB <= 16)) {
    const double rows = g.npad - g.c0;
    trace::Scope ts(st, EXPM_PFD_K_PANEL, (double)P * 4.0 * rows * IB * IB,
                    (double)P * 2.0 * rows * IB * sizeof(cx<R>));
    hipLaunchKernelGGL((k_panel<R, IB, S>), dim3(P), dim3(PANEL_NT), 0, st, W, g.ws, g.ld, g.npad, g.j0, g.c0, g.nbo,
                       g.ipiv, g.ps, g.moves, g.ms, g.step, g.last);
  }
}

template <typename R, int IB>
void panel_dispatch(hipStream_t st, int S, const PanelArgs& g, cx<R>* W) {
  switch (S) {
#define CASE(s)                                   \
  case s:                                         \
    panel_launch<R, IB, s>(st, g, W); \
    break;
    CASE(1)
    CASE(2)
    CASE(3)
    CASE(4)
    CASE(5)
    CASE(6)
    CASE(7)
    CASE(8)
    CASE(9)
    CASE(10)
    CASE(11)
    CASE(12)
    CASE(13)
    CASE(14)
    CASE(15)
    CASE(16)
#undef CASE
    default:
      break;
  }
}

template <typename R>
void panel(hipStream_t st, int IB, int S, const PanelArgs& g, cx<R>* W) {
  switch (IB) {
    case 16:
      panel_dispatch<R, 16>(st, S, g, W);
      break;
    case 8:
      panel_dispatch<R, 8>(st, S, g, W);
      break;
    case 4:
      panel_dispatch<R, 4>(st, S, g, W);
      break;
    default:
      panel_dispatch<R, 2>(st, S, g, W);
      break;
  }
}

// Tile shapes of the LU trailing update (C -= L21 U12 over the whole trailing
// matrix).  Every shape runs the same K loop per output element (same chunk
// order, same matrix-core instruction), so the choice never changes a bit of
// the result; it is a speed knob only (built-in: 64 x 64; the autotuner times
// all of them).
constexpr int LU_TILES = LU_TILE_COUNT;
const char* const LU_TILE_NAMES[LU_TILES] = {"64x64", "128x64", "64x128"};

// The plain and (GATABLE) the gated kernel of one k_gemm instantiation.
template <typename R, int MODE, int BM, int BN, int WGM, int WGN, int TAG = 0, bool GATABLE = true>
struct GemmKernels {
  static constexpr bool gatable = GATABLE;
  static constexpr auto plain = &k_gemm<R, MODE, BM, BN, WGM, WGN, TAG>;
  static constexpr auto gated = &k_gemm_gated<R, MODE, BM, BN, WGM, WGN, TAG>;
};

// MODE 0: C -= op(A) B;  MODE 1: C = op(A) B.  Batches < split use a0, others a1.
// tile: LU trailing-update shape (index into LU_TILE_NAMES), MODE 0 only.
// gate: non-null for products of refinement sweeps (skipped once *gate == 0).
template <typename R, int MODE>
void gemm(hipStream_t st, int cls, int batch, int M, int N, int K, GemmOperand<R> a0, GemmOperand<R> a1, int split,
          const cx<R>* B, int64_t sB, int64_t ldb, cx<R>* C, int64_t sC, int64_t ldc, KSplit ksp = {1, 0, 0, 0},
          int tile = 0, const int* gate = nullptr) {
  if (M <= 0 || N <= 0 || K <= 0 || batch <= 0) return;
  const double e = sizeof(cx<R>);
  const double Kt = (double)K * ksp.ks;
  trace::Scope ts(st, cls, 8.0 * batch * (double)M * N * Kt,
                  e * batch * ((double)M * Kt + Kt * N + (MODE == 0 ? 2.0 : (double)ksp.ks) * M * N), true);
  const unsigned gy = (unsigned)(batch * ksp.ks);
  auto launch = [&](auto kernels, dim3 grid) {
    using K2 = decltype(kernels);
    if constexpr (K2::gatable) {
      if (gate != nullptr) {
        if (ts.active)
          hipExtLaunchKernelGGL(K2::gated, grid, dim3(256), 0, st, ts.r.a, ts.r.b, 0, gate, M, N, K, a0, a1, split,
                                B, sB, ldb, C, sC, ldc, ksp);
        else
          hipLaunchKernelGGL(K2::gated, grid, dim3(256), 0, st, gate, M, N, K, a0, a1, split, B, sB, ldb, C, sC, ldc,
                             ksp);
        return;
      }
    }
    if (ts.active) {
      hipExtLaunchKernelGGL(K2::plain, grid, dim3(256), 0, st, ts.r.a, ts.r.b, 0, M, N, K, a0, a1, split, B, sB,
                            ldb, C, sC, ldc, ksp);
    } else {
      hipLaunchKernelGGL(K2::plain, grid, dim3(256), 0, st, M, N, K, a0, a1, split, B, sB, ldb, C, sC, ldc, ksp);
    }
  };
  if (N <= 16 && cls != EXPM_PFD_K_LU_GEMM && cls != EXPM_PFD_K_LU_TRAIL && cls != EXPM_PFD_K_LU_TRSM) {
    launch(GemmKernels<R, MODE, 64, 16, 4, 1>{}, dim3((unsigned)((M + 63) / 64), gy));
    return;
  }
  // whole-tile products with one unconjugated operand (LU updates and U12, the
  // refinement product, the block products of wide solves): their own
  // instantiation, same bits as the general one
  if ((cls == EXPM_PFD_K_LU_GEMM || cls == EXPM_PFD_K_LU_TRSM || cls == EXPM_PFD_K_IR_GEMM ||
       cls == EXPM_PFD_K_SOLVE_GEMM) &&
      M % 64 == 0 && N % 64 == 0 && K % 16 == 0 && a0.conj == 0 && split >= batch) {
    launch(GemmKernels<R, MODE, 64, 64, 2, 2, 2>{}, dim3((unsigned)((M / 64) * (N / 64)), gy));
    return;
  }
  if constexpr (MODE == 0) {
    const bool trail = cls == EXPM_PFD_K_LU_TRAIL && K % 16 == 0 && a0.conj == 0;
    if (tile == 1) {
      if (trail && M % 128 == 0 && N % 64 == 0)
        launch(GemmKernels<R, MODE, 128, 64, 2, 2, 1, false>{}, dim3((unsigned)((M / 128) * (N / 64)), gy));
      else
        launch(GemmKernels<R, MODE, 128, 64, 2, 2, 0, false>{},
               dim3((unsigned)(((M + 127) / 128) * ((N + 63) / 64)), gy));
      return;
    }
    if (tile == 2) {
      if (trail && M % 64 == 0 && N % 128 == 0)
        launch(GemmKernels<R, MODE, 64, 128, 2, 2, 1, false>{}, dim3((unsigned)((M / 64) * (N / 128)), gy));
      else
        launch(GemmKernels<R, MODE, 64, 128, 2, 2, 0, false>{},
               dim3((unsigned)(((M + 63) / 64) * ((N + 127) / 128)), gy));
      return;
    }
    // the trailing update's own instantiation needs whole tiles and chunks (always
    // so: padded orders and panel widths are multiples of 64); otherwise the general one
    if (cls == EXPM_PFD_K_LU_TRAIL && M % 64 == 0 && N % 64 == 0 && K % 16 == 0 && a0.conj == 0) {
      launch(GemmKernels<R, MODE, 64, 64, 2, 2, 1, false>{},
             dim3((unsigned)(((M + 63) / 64) * ((N + 63) / 64)), gy));
      return;
    }
  }
  launch(GemmKernels<R, MODE, 64, 64, 2, 2>{}, dim3((unsigned)(((M + 63) / 64) * ((N + 63) / 64)), gy));
}

// K slices of the FP64 refinement product (t A) X for thin right-hand sides: a
// function of the padded order only, so a problem's bits do not depend on the
// batch it runs in
inline int ir_kslices(int64_t npad) {
  int s = 1;
  while (s < 8 && npad / (2 * s) >= 256) s *= 2;
  return s;
}

template <typename R>
GemmOperand<R> opnd(const cx<R>* p, int64_t stride, int64_t ld, bool conj) {
  GemmOperand<R> o;
  o.p = p;
  o.stride = stride;
  o.ld = ld;
  o.conj = conj ? 1 : 0;
  return o;
}

// gate: see KSplit (nullptr: always runs)
template <typename R>
void moves_apply(hipStream_t st, int batch, cx<R>* Bm, int64_t sB, int64_t ldb, int ncols, int gap_at, int gap_len,
                 const int* moves, int64_t smv, int s_begin, int s_end, int inverse, const int* gate = nullptr) {
  if (ncols <= 0 || s_end <= s_begin) return;
  trace::Scope ts(st, EXPM_PFD_K_MOVES, 0.0, 0.0);
  const int g = (ncols + 15) / 16;
  hipLaunchKernelGGL((k_moves<R, 16>), dim3(g, batch), dim3(256), 0, st, Bm, sB, ldb, ncols, gap_at, gap_len, moves,
                     smv, s_begin, s_end, inverse, gate);
}

// which: 0 = L11^{-1}, 1 = U11^{-1}, 2 = both, for steps [step0, step0 + nsteps)
template <typename R>
void block_inverse(hipStream_t st, int batch, const cx<R>* W, int64_t ws, int64_t ld, int step0, int nsteps,
                   int which, cx<R>* dinv, int64_t ds) {
  if (nsteps <= 0) return;
  const int nmat = which == 2 ? 2 : 1;
  trace::Scope ts(st, EXPM_PFD_K_PANEL, 8.0 * batch * nsteps * nmat * NB * NB * NB / 6.0,
                  sizeof(cx<R>) * 2.0 * batch * nsteps * nmat * NB * NB);
  // one 16-wave workgroup per block once a launch has enough blocks to fill the
  // device; otherwise four 4-wave workgroups per block (same bits either way)
  if ((int64_t)batch * nmat * nsteps >= 256)
    hipLaunchKernelGGL((k_block_inverse<R, 16>), dim3(nmat * nsteps, batch), dim3(64 * 16), 0, st, W, ws, ld, step0,
                       which, dinv, ds);
  else
    hipLaunchKernelGGL((k_block_inverse<R, 4>), dim3(4 * nmat * nsteps, batch), dim3(64 * 4), 0, st, W, ws, ld, step0,
                       which, dinv, ds);
}

// One factorization step's interchanges on the columns outside its panel, then
// (with linv) the inverse of its L11.  Where the inverse runs as four 4-wave
// workgroups per matrix, both go into one launch (k_moves_inverse): they touch
// disjoint data, and the two short launches cost more apart than together.
template <typename R>
void moves_and_linv(hipStream_t st, int batch, cx<R>* W, int64_t ws, int64_t ld, int ncols, int gap_at, int gap_len,
                    const int* mv, int64_t smv, int step, bool linv, cx<R>* dinv, int64_t ds) {
  if (!linv || ncols <= 0 || batch >= 256) {
    moves_apply<R>(st, batch, W, ws, ld, ncols, gap_at, gap_len, mv, smv, 0, 1, 0);
    if (linv) block_inverse<R>(st, batch, W, ws, ld, step, 1, 0, dinv, ds);
    return;
  }
  // FP64: the inverse's LDS leaves two workgroups per CU, so wider column groups
  // keep the moves to one round of workgroups
  constexpr int CW = sizeof(R) == 8 ? 64 : 32;
  const int gm = (ncols + CW - 1) / CW;
  trace::Scope ts(st, EXPM_PFD_K_PANEL, 8.0 * batch * NB * NB * NB / 6.0, sizeof(cx<R>) * 2.0 * batch * NB * NB);
  hipLaunchKernelGGL((k_moves_inverse<R, CW>), dim3(gm + 4, batch), dim3(256), 0, st, W, ws, ld, ncols, gap_at,
                     gap_len, mv, smv, gm, step, dinv, ds);
}

inline int grid_for(int64_t count) {
  int64_t g = (count + 255) / 256;
  return (int)std::min<int64_t>(std::max<int64_t>(g, 1), 65536);
}

}  // namespace

// ============================================================================
// plan: workspace for G problems of the same padded order (G = 1 for
// expm_pfd_plan; groups of the batched entry point use G > 1).  Every launch of
// the factorization and the solves covers all G*P shifted matrices.
// ============================================================================
struct expm_pfd_plan_s {
  int64_t n = 0, npad = 0, m_max = 0;  // n, m_max: the single-problem arguments
  int G = 1, degree = 0, P = 0, PB = 0, precision = EXPM_PFD_FP64, ir_sweeps = 2, IB = 16, nsteps = 0;
  int ir_ext = 0;  // last sweeps with double-double residuals
  double ir_tol = 1e-10;  // convergence test of the refinement (< 0: none, fixed sweep count)
  double shift = 0.0;     // c of the shifting method (tA units, or A units with shift_t)
  int shift_t = 0;        // the shift is in units of A: problem i uses t_i * shift
  int real_data = 0;  // A and V real: conjugate poles need no solves of their own
  int upper = 0;      // the upper triangle of A is read
  int Gcap = 1;  // problems the workspace was sized for; G <= Gcap is the active count
  double t = 1;
  bool full_ok = false;
  int64_t mp_max = 16, cols_alloc = 0;
  std::vector<double2> h_theta, h_a;
  double2* d_theta = nullptr;
  double2* d_a = nullptr;
  void* W = nullptr;         // PB x npad x npad, FP64 or FP32 complex, row-major
  int* ipiv = nullptr;       // PB x npad
  int* moves = nullptr;      // PB x nsteps x MOVE_STRIDE
  void* dinv = nullptr;      // PB x nsteps x 2 x 64 x 64: inverses of the diagonal blocks of L and U
  // one-launch sweeps: the control line (ticket and finish counters, status,
  // epoch: SW_*), then from int FLAG_STRIDE on 2PB x chains x nsteps ready flags,
  // FLAG_STRIDE ints apart.  Kept on the device only, so sweeps replay in graphs.
  int* sweep_sync = nullptr;
  void* Xs = nullptr;        // npad x cols_alloc, working type
  double2* Ah = nullptr;     // mixed: G x npad x npad FP64 t*A (Hermitian, row-major)
  double2* X64 = nullptr;    // mixed: npad x cols_alloc
  double2* R64 = nullptr;    // mixed: npad x cols_alloc
  double2* Rpart = nullptr;  // mixed: ir_kslices(npad) x npad x (2 PB min(mp_max, 64)) split-K partials
  int* ir_words = nullptr;   // mixed: [0] refinement gate, [1] the check's finish counter, [2 + g] problem
                             // g's solves missed ir_tol (g < G), then one convergence word per block
  unsigned long long* ir_max = nullptr;  // mixed: 2 x 2PB per-block maxima of the convergence test
  ProblemDesc* d_descs = nullptr;  // G problem descriptors on the device (batched entry point)
  int device = 0;
  bool pooled = false;             // workspace from the stream-ordered pool (freed on `pool`)
  hipStream_t pool = nullptr;
  int lu_tile = 0;                 // LU trailing-update tile shape (LU_TILE_NAMES)
  int use_graph = 0;               // expm_pfd_apply replays captured graphs
  hipStream_t cap = nullptr;       // stream the graphs are captured on (plan-owned)
  std::map<std::pair<int, int64_t>, hipGraphExec_t> graphs;  // (V = I, m) -> executable graph
};

namespace {

struct Sizes {
  int64_t npad, cols, w_elem;
  size_t w, ipiv, moves, dinv, sweep, xs, ah, x64, r64, rpart, consts, descs, irw, irm;
  size_t total() const {
    return w + ipiv + moves + dinv + sweep + xs + ah + x64 + r64 + rpart + consts + descs + irw + irm;
  }
};

Sizes plan_sizes(int64_t npad, int G, int degree, int64_t mp_max, bool full_ok, int precision) {
  Sizes s{};
  const int64_t PB = (int64_t)G * (degree / 2);
  s.npad = npad;
  s.cols = std::max<int64_t>(full_ok ? PB * npad : 0, 2 * PB * mp_max);
  const bool fp64 = precision == EXPM_PFD_FP64;
  s.w_elem = fp64 ? 16 : 8;
  s.w = (size_t)PB * npad * npad * s.w_elem;
  s.ipiv = (size_t)PB * npad * sizeof(int);
  s.moves = (size_t)PB * (npad / NB) * MOVE_STRIDE * sizeof(int);
  s.dinv = (size_t)PB * (npad / NB) * 2 * NB * NB * s.w_elem;
  s.sweep = (size_t)(FLAG_STRIDE + 2 * PB * (CHAIN_MP_MAX / 16) * (npad / NB) * FLAG_STRIDE) * sizeof(int);
  s.xs = (size_t)npad * s.cols * s.w_elem;
  s.ah = fp64 ? 0 : (size_t)G * npad * npad * 16;
  s.x64 = fp64 ? 0 : (size_t)npad * s.cols * 16;
  s.r64 = s.x64;
  s.rpart = fp64 ? 0 : (size_t)ir_kslices(npad) * npad * (2 * PB * std::min<int64_t>(mp_max, CHAIN_MP_MAX)) * 16;
  s.consts = 2 * 64 * 16;
  s.descs = (size_t)G * sizeof(ProblemDesc);
  s.irw = fp64 ? 0 : (size_t)(2 + G + 2 * PB) * sizeof(int);
  // two per workgroup of the per-block refinement kernels (at most max(2048, 2 PB) workgroups)
  s.irm = fp64 ? 0 : (size_t)2 * std::max<int64_t>(2048, 2 * PB) * sizeof(unsigned long long);
  return s;
}

void free_plan(expm_pfd_plan_t p) {
  if (!p) return;
  for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  void* ptrs[] = {p->d_theta, p->d_a, p->W,     p->ipiv,    p->moves,    p->dinv,  p->sweep_sync, p->Xs,
                  p->Ah,      p->X64, p->R64,   p->Rpart,   p->d_descs, p->ir_words, p->ir_max};
  for (void* q : ptrs)
    if (q) (void)(p->pooled ? hipFreeAsync(q, p->pool) : hipFree(q));
  delete p;
}

// sticky fault bits of the plan's one-launch sweeps (0: every wait ended in order);
// call once the plan's work has completed
int sweep_fault(expm_pfd_plan_t p) {
  int f = 0;
  if (hipMemcpy(&f, p->sweep_sync + SW_STATUS, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return -1;
  return f;
}

// Where a plan's workspace comes from: hipMalloc (pool == nullptr), or the
// device's stream-ordered pool on stream pool->s (fast once the pool holds
// memory: the serving queue and one-shot batches create plans while other
// work runs).
struct PoolArg {
  hipStream_t s;
};

// Freed blocks of the default stream-ordered pool stay in it for reuse (once
// per device; idempotent).
void keep_pool_memory(int device) {
  hipMemPool_t mpool = nullptr;
  if (hipDeviceGetDefaultMemPool(&mpool, device) == hipSuccess) {
    uint64_t keep = UINT64_MAX;
    (void)hipMemPoolSetAttribute(mpool, hipMemPoolAttrReleaseThreshold, &keep);
  }
  (void)hipGetLastError();
}

// Poles and residues of the plan: one member per conjugate pair (Im theta > 0).
// The shifting method of Remark rem:shift,
//   e^c R_d(tA - cI) = sum_k (e^c a_k) (tA + (theta_k - c) I)^{-1},
// is applied per problem by the kernels (ProblemDesc::c, ::ec).
int pole_constants(int degree, double2* theta, double2* a) {
  return expm_pfd_constants(degree, (double*)theta, (double*)a);
}

// The plan's scalar fields for G problems of padded order npad (everything but
// the constants and the device pointers).
void init_plan_fields(expm_pfd_plan_s* pl, int64_t npad, int G, int degree, int64_t mp_max, bool full_ok,
                      int precision, int ir_max_iter, int ir_extended, int real_data, double ir_tol) {
  pl->G = G;
  pl->Gcap = G;
  pl->degree = degree;
  pl->P = degree / 2;
  pl->PB = G * pl->P;
  pl->precision = precision;
  // degree >= 32: one more sweep, the last with a double-double residual
  pl->ir_sweeps = ir_max_iter > 0 ? ir_max_iter : ir_max_iter < 0 ? 0 : degree >= 32 ? 3 : 2;
  pl->ir_tol = ir_tol == 0.0 ? 1e-10 : ir_tol;
  pl->real_data = real_data ? 1 : 0;
  pl->ir_ext = std::min(pl->ir_sweeps, ir_extended < 0 ? 0 : ir_extended > 0 ? ir_extended : degree >= 32 ? 1 : 0);
  pl->full_ok = full_ok;
  pl->mp_max = mp_max;
  pl->npad = npad;
  pl->nsteps = (int)(npad / NB);
  pl->cols_alloc = plan_sizes(npad, G, degree, mp_max, full_ok, precision).cols;
  pl->IB = inner_width(npad, precision == EXPM_PFD_FP64);
}

// opts: the options that shape the plan's work (precision excepted): refinement
// sweeps, tolerance and extended sweeps, real data, shift (NULL: defaults)
int create_plan(expm_pfd_plan_t* out, int64_t npad, int G, int degree, int64_t mp_max, bool full_ok, int precision,
                const expm_pfd_opts* opts, const PoolArg* pool = nullptr) {
  auto* pl = new expm_pfd_plan_s();
  pl->pooled = pool != nullptr;
  pl->pool = pool ? pool->s : nullptr;
  init_plan_fields(pl, npad, G, degree, mp_max, full_ok, precision, opts ? opts->ir_max_iter : 0,
                   opts ? opts->ir_extended : 0, opts ? opts->real_data : 0, opts ? opts->ir_tol : 0.0);
  pl->shift = opts ? opts->shift : 0.0;
  pl->shift_t = opts && opts->shift_scale_t ? 1 : 0;
  const Sizes sz = plan_sizes(npad, G, degree, mp_max, full_ok, precision);
  pl->h_theta.resize(pl->P);
  pl->h_a.resize(pl->P);
  int rc = pole_constants(degree, pl->h_theta.data(), pl->h_a.data());
  if (rc) {
    delete pl;
    return rc;
  }
  (void)hipGetDevice(&pl->device);
  HipErr he;
  auto dmalloc = [&](auto** p, size_t bytes) {
    he(pool ? hipMallocAsync((void**)p, bytes, pool->s) : hipMalloc((void**)p, bytes));
  };
  dmalloc(&pl->d_theta, 64 * sizeof(double2));
  dmalloc(&pl->d_a, 64 * sizeof(double2));
  dmalloc(&pl->W, sz.w);
  dmalloc(&pl->ipiv, sz.ipiv);
  dmalloc(&pl->moves, sz.moves);
  dmalloc(&pl->dinv, sz.dinv);
  dmalloc(&pl->sweep_sync, sz.sweep);
  dmalloc(&pl->Xs, sz.xs);
  dmalloc(&pl->d_descs, sz.descs);
  if (precision == EXPM_PFD_MIXED) {
    dmalloc(&pl->Ah, sz.ah);
    dmalloc(&pl->X64, sz.x64);
    dmalloc(&pl->R64, sz.r64);
    dmalloc(&pl->Rpart, sz.rpart);
    dmalloc(&pl->ir_words, sz.irw);
    dmalloc(&pl->ir_max, sz.irm);
  }
  if (he.e == hipSuccess && pool) {
    // the constants' host copies live in the plan, so the copies may complete later
    he(hipMemcpyAsync(pl->d_theta, pl->h_theta.data(), pl->P * sizeof(double2), hipMemcpyHostToDevice, pool->s));
    he(hipMemcpyAsync(pl->d_a, pl->h_a.data(), pl->P * sizeof(double2), hipMemcpyHostToDevice, pool->s));
    he(hipMemsetAsync(pl->moves, 0, sz.moves, pool->s));
    he(hipMemsetAsync(pl->sweep_sync, 0, sz.sweep, pool->s));
  } else if (he.e == hipSuccess) {
    he(hipMemcpy(pl->d_theta, pl->h_theta.data(), pl->P * sizeof(double2), hipMemcpyHostToDevice));
    he(hipMemcpy(pl->d_a, pl->h_a.data(), pl->P * sizeof(double2), hipMemcpyHostToDevice));
    he(hipMemset(pl->moves, 0, sz.moves));
    he(hipMemset(pl->sweep_sync, 0, sz.sweep));
  }
  if (he.e != hipSuccess) {
    const bool oom = he.e == hipErrorOutOfMemory;
    (void)hipGetLastError();
    free_plan(pl);
    return oom ? EXPM_PFD_ERR_OOM : EXPM_PFD_ERR_HIP;
  }
  *out = pl;
  return 0;
}

// ---- graphs ------------------------------------------------------------------------
// Captures the work fn(stream) enqueues on `cap` into an executable graph.
template <typename F>
int capture_graph(hipStream_t cap, F&& fn, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  *out = nullptr;
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return EXPM_PFD_ERR_HIP;
  int rc = fn(cap);
  if (hipStreamEndCapture(cap, &g) != hipSuccess && rc == 0) rc = EXPM_PFD_ERR_HIP;
  if (rc == 0 && hipGraphInstantiate(out, g, nullptr, nullptr, 0) != hipSuccess) {
    *out = nullptr;
    rc = EXPM_PFD_ERR_HIP;
  }
  if (g) (void)hipGraphDestroy(g);
  (void)hipGetLastError();
  return rc;
}

int ensure_capture_stream(expm_pfd_plan_t pl) {
  if (pl->cap) return 0;
  return hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking) == hipSuccess ? 0 : EXPM_PFD_ERR_HIP;
}

// ---- autotuner -----------------------------------------------------------------------
// Times every LU trailing-update tile shape on the plan's first two-step update
// (M = N = npad - 128, K = 128, all PB shifted matrices) and returns the
// fastest.  The shapes give bitwise-identical results, so the choice only
// affects speed.  Choices are cached per (padded order, precision, batch).
std::mutex tune_mu;
std::map<std::tuple<int64_t, int, int>, int> tune_cache;

template <typename R>
int tune_lu_tile_t(expm_pfd_plan_t pl) {
  const int npad = (int)pl->npad, PB = pl->PB;
  const int K = pl->nsteps >= 2 ? 2 * NB : NB;
  const int M = npad - K;
  if (M < NB || ensure_capture_stream(pl)) return 0;
  hipStream_t s = pl->cap;
  const int64_t ld = npad, ws = (int64_t)npad * npad;
  cx<R>* W = (cx<R>*)pl->W;
  if (hipMemsetAsync(pl->W, 0, (size_t)PB * ws * sizeof(cx<R>), s) != hipSuccess) return 0;
  const unsigned saved = trace::mask;
  trace::mask = 0;
  hipEvent_t a = nullptr, b = nullptr;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  int best = 0;
  float best_ms = 0.f;
  for (int tile = 0; tile < LU_TILES; ++tile) {
    auto once = [&] {
      gemm<R, 0>(s, EXPM_PFD_K_LU_TRAIL, PB, M, M, K, opnd<R>(W + (int64_t)K * ld, ws, ld, false),
                 opnd<R>(nullptr, 0, 0, false), PB, W + K, ws, ld, W + (int64_t)K * ld + K, ws, ld, {1, 0, 0, 0},
                 tile);
    };
    once();
    (void)hipEventRecord(a, s);
    for (int r = 0; r < 3; ++r) once();
    (void)hipEventRecord(b, s);
    float ms = 0.f;
    if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess) break;
    if (tile == 0 || ms < best_ms) {
      best = tile;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  trace::mask = saved;
  (void)hipGetLastError();
  return best;
}

int tune_lu_tile(expm_pfd_plan_t pl) {
  const auto key = std::make_tuple(pl->npad, pl->precision, pl->PB);
  {
    std::lock_guard<std::mutex> lk(tune_mu);
    auto it = tune_cache.find(key);
    if (it != tune_cache.end()) return it->second;
  }
  const int t = pl->precision == EXPM_PFD_FP64 ? tune_lu_tile_t<double>(pl) : tune_lu_tile_t<float>(pl);
  std::lock_guard<std::mutex> lk(tune_mu);
  tune_cache[key] = t;
  return t;
}

// Options that do not change the workspace: tile shape and graph replay.
int configure_plan(expm_pfd_plan_t pl, const expm_pfd_opts* o) {
  if (!o) return 0;
  pl->use_graph = o->graph ? 1 : 0;
  if (o->lu_tile > 0)
    pl->lu_tile = o->lu_tile - 1;
  else if (o->autotune)
    pl->lu_tile = tune_lu_tile(pl);
  if (pl->use_graph) return ensure_capture_stream(pl);
  return 0;
}

// ---- factorization of all shifted matrices of the group --------------------------
// Panel phase of outer step `step` (columns [j0, j0+nbo)): the inner register
// panels and the updates inside the outer panel.
template <typename R>
void panel_phase(expm_pfd_plan_t pl, int step, hipStream_t st) {
  const int PB = pl->PB, npad = (int)pl->npad;
  const int64_t ld = npad, ws = (int64_t)npad * npad;
  const int64_t mstride = (int64_t)pl->nsteps * MOVE_STRIDE;
  cx<R>* W = (cx<R>*)pl->W;
  const int j0 = step * NB, nbo = std::min(NB, npad - j0);
  const int IB = inner_width_at(pl->IB, npad - j0, sizeof(R) == 8);
  for (int c0 = j0; c0 < j0 + nbo; c0 += IB) {
    PanelArgs g;
    g.ws = ws;
    g.ld = ld;
    g.ps = npad;
    g.ms = mstride;
    g.P = PB;
    g.npad = npad;
    g.j0 = j0;
    g.c0 = c0;
    g.nbo = nbo;
    g.step = step;
    g.last = (c0 + IB >= j0 + nbo);
    g.ipiv = pl->ipiv;
    g.moves = pl->moves;
    panel<R>(st, IB, (npad - c0 + PANEL_NT - 1) / PANEL_NT, g, W);
    const int rest = j0 + nbo - c0 - IB;
    if (rest > 0) {
      const int64_t r1 = c0 + IB;
      gemm<R, 0>(st, EXPM_PFD_K_LU_GEMM, PB, npad - c0 - IB, rest, IB, opnd<R>(W + r1 * ld + c0, ws, ld, false),
                 opnd<R>(nullptr, 0, 0, false), PB, W + (int64_t)c0 * ld + r1, ws, ld, W + r1 * ld + r1, ws, ld);
    }
  }
}

// After the panel phase of `step`: its interchanges on the other columns, the
// L11 inverse, U12 = L11^{-1} A12 and the trailing update A22 -= L21 U12.
template <typename R>
void step_update(expm_pfd_plan_t pl, int step, hipStream_t st) {
  const int PB = pl->PB, npad = (int)pl->npad;
  const int64_t ld = npad, ws = (int64_t)npad * npad;
  const int64_t ds = (int64_t)pl->nsteps * 2 * NB * NB;
  const int64_t mstride = (int64_t)pl->nsteps * MOVE_STRIDE;
  cx<R>* W = (cx<R>*)pl->W;
  cx<R>* dinv = (cx<R>*)pl->dinv;
  const int j0 = step * NB, nbo = std::min(NB, npad - j0);
  const int* mv = pl->moves + (int64_t)step * MOVE_STRIDE;
  const int ntr = npad - j0 - nbo;
  moves_and_linv<R>(st, PB, W, ws, ld, j0 + ntr, j0, nbo, mv, mstride, step, ntr > 0, dinv, ds);
  if (ntr <= 0) return;
  const int64_t c1 = j0 + nbo;
  const cx<R>* Linv = dinv + (int64_t)step * 2 * NB * NB;
  gemm<R, 1>(st, EXPM_PFD_K_LU_TRSM, PB, nbo, ntr, nbo, opnd<R>(Linv, ds, NB, false), opnd<R>(nullptr, 0, 0, false),
             PB, W + (int64_t)j0 * ld + c1, ws, ld, W + (int64_t)j0 * ld + c1, ws, ld);
  gemm<R, 0>(st, EXPM_PFD_K_LU_TRAIL, PB, ntr, ntr, nbo, opnd<R>(W + c1 * ld + j0, ws, ld, false),
             opnd<R>(nullptr, 0, 0, false), PB, W + (int64_t)j0 * ld + c1, ws, ld, W + c1 * ld + c1, ws, ld,
             {1, 0, 0, 0}, pl->lu_tile);
}

// Two steps j, j+1 with one trailing update of depth 2 NB.  Step j's update is
// applied at once only where step j+1 needs it: the columns of panel j+1 (before
// that panel is factored) and the rows of U12 of step j+1 (before it is formed).
// The rest of the trailing matrix gets both steps' updates from one product,
// A22 -= [L21_j L21_j+1] [U12_j; U12_j+1], which reads and writes A22 once per
// two steps.  Step j+1's interchanges reach the rows still waiting for step j's
// update together with the rows of L21_j (the left columns), so the deferred
// product stays consistent; in exact arithmetic the factors are those of the
// one-step order.
template <typename R>
void step_pair(expm_pfd_plan_t pl, int step, hipStream_t st) {
  const int PB = pl->PB, npad = (int)pl->npad;
  const int64_t ld = npad, ws = (int64_t)npad * npad;
  const int64_t ds = (int64_t)pl->nsteps * 2 * NB * NB;
  const int64_t mstride = (int64_t)pl->nsteps * MOVE_STRIDE;
  cx<R>* W = (cx<R>*)pl->W;
  cx<R>* dinv = (cx<R>*)pl->dinv;
  const int64_t j0 = (int64_t)step * NB, c1 = j0 + NB;
  const int nb2 = std::min<int>(NB, npad - (int)c1);
  const int64_t c2 = c1 + nb2;
  const int ntr1 = npad - (int)c1, ntr2 = npad - (int)c2;
  // step j: panel, its interchanges elsewhere, L11^{-1}, U12 over every right column
  panel_phase<R>(pl, step, st);
  moves_and_linv<R>(st, PB, W, ws, ld, (int)j0 + ntr1, (int)j0, NB, pl->moves + (int64_t)step * MOVE_STRIDE, mstride,
                    step, true, dinv, ds);
  gemm<R, 1>(st, EXPM_PFD_K_LU_TRSM, PB, NB, ntr1, NB, opnd<R>(dinv + (int64_t)step * 2 * NB * NB, ds, NB, false),
             opnd<R>(nullptr, 0, 0, false), PB, W + j0 * ld + c1, ws, ld, W + j0 * ld + c1, ws, ld);
  // step j's update of the columns of panel j+1
  gemm<R, 0>(st, EXPM_PFD_K_LU_GEMM, PB, ntr1, nb2, NB, opnd<R>(W + c1 * ld + j0, ws, ld, false),
             opnd<R>(nullptr, 0, 0, false), PB, W + j0 * ld + c1, ws, ld, W + c1 * ld + c1, ws, ld);
  // step j+1: panel and its interchanges on the columns left and right of it
  panel_phase<R>(pl, step + 1, st);
  moves_and_linv<R>(st, PB, W, ws, ld, (int)c1 + ntr2, (int)c1, nb2, pl->moves + (int64_t)(step + 1) * MOVE_STRIDE,
                    mstride, step + 1, ntr2 > 0, dinv, ds);
  if (ntr2 <= 0) return;
  // step j's update of the rows of U12_j+1, then U12_j+1 = L11^{-1} A12
  gemm<R, 0>(st, EXPM_PFD_K_LU_GEMM, PB, nb2, ntr2, NB, opnd<R>(W + c1 * ld + j0, ws, ld, false),
             opnd<R>(nullptr, 0, 0, false), PB, W + j0 * ld + c2, ws, ld, W + c1 * ld + c2, ws, ld);
  gemm<R, 1>(st, EXPM_PFD_K_LU_TRSM, PB, nb2, ntr2, nb2,
             opnd<R>(dinv + (int64_t)(step + 1) * 2 * NB * NB, ds, NB, false), opnd<R>(nullptr, 0, 0, false), PB,
             W + c1 * ld + c2, ws, ld, W + c1 * ld + c2, ws, ld);
  // both steps' update of the trailing matrix
  gemm<R, 0>(st, EXPM_PFD_K_LU_TRAIL, PB, ntr2, ntr2, NB + nb2, opnd<R>(W + c2 * ld + j0, ws, ld, false),
             opnd<R>(nullptr, 0, 0, false), PB, W + j0 * ld + c2, ws, ld, W + c2 * ld + c2, ws, ld, {1, 0, 0, 0},
             pl->lu_tile);
}

template <typename R>
void factor(expm_pfd_plan_t pl, const ProblemDesc* descs, const ProblemDesc& one, hipStream_t st) {
  const int P = pl->P, PB = pl->PB;
  const int npad = (int)pl->npad;
  const int64_t ld = npad, ws = (int64_t)npad * npad;
  cx<R>* W = (cx<R>*)pl->W;
  {
    dim3 g(npad / 32, npad / 32, pl->G), b(32, 8);
    trace::Scope ts(st, EXPM_PFD_K_FORM, 0.0,
                    (double)pl->G * npad * npad * 16 + (double)PB * npad * npad * sizeof(cx<R>) +
                        (pl->Ah ? (double)pl->G * npad * npad * 16 : 0.0));
    hipLaunchKernelGGL((k_form<R>), g, b, 0, st, descs, one, npad, pl->d_theta, P, W, ws, ld, pl->Ah, (int64_t)npad);
  }
  cx<R>* dinv = (cx<R>*)pl->dinv;
  const int64_t ds = (int64_t)pl->nsteps * 2 * NB * NB;
  const int nsteps = pl->nsteps;
  // (overlapping the panels of step j+1 with the update of step j on two streams,
  // with or without CUs kept free for the panels, measured slower on gfx950)
  int step = 0;
  for (; step + 1 < nsteps; step += 2) step_pair<R>(pl, step, st);
  if (step < nsteps) {
    panel_phase<R>(pl, step, st);
    step_update<R>(pl, step, st);
  }
  // diagonal-block inverses still missing for the sweeps: every U11, the last L11
  block_inverse<R>(st, PB, W, ws, ld, 0, nsteps, 1, dinv, ds);
  block_inverse<R>(st, PB, W, ws, ld, nsteps - 1, 1, 0, dinv, ds);
}

// ---- solves on all right-hand-side blocks ----------------------------------------
// Blocks [0, PB) hold primal right-hand sides (shifted matrix b), blocks [PB, 2PB)
// (if adjoint) the conjugate-pole ones; each block is mp columns of the
// row-major npad x ldS array X.
template <typename R>
SweepOperand<R> sweep_op(const cx<R>* p, int64_t stride, int64_t ld, bool conj) {
  SweepOperand<R> o;
  o.p = p;
  o.stride = stride;
  o.ld = ld;
  o.conj = conj ? 1 : 0;
  return o;
}

// Thin right-hand sides (mp <= CHAIN_MP_MAX): each sweep is one launch in which
// every 16-column chain runs its block steps back to back (k_sweep_chain).
template <typename R>
void solves_chain(expm_pfd_plan_t pl, cx<R>* X, int64_t ldS, int mp, bool adjoint, hipStream_t st,
                  const int* gate) {
  const int PB = pl->PB;
  const int npad = (int)pl->npad;
  const int64_t ld = npad, ws = (int64_t)npad * npad;
  const cx<R>* W = (const cx<R>*)pl->W;
  const cx<R>* dinv = (const cx<R>*)pl->dinv;
  const int64_t ds = (int64_t)pl->nsteps * 2 * NB * NB;
  const int64_t mstride = (int64_t)pl->nsteps * MOVE_STRIDE;
  const int nsteps = pl->nsteps;
  const int nblk = adjoint ? 2 * PB : PB;
  const int cpb = mp / 16, nchain = nblk * cpb;
  const double e = sizeof(cx<R>);
  moves_apply<R>(st, PB, X, mp, ldS, mp, mp, 0, pl->moves, mstride, 0, nsteps, 0, gate);
  for (int dirn = 0; dirn < 2; ++dirn) {
    const bool fwd = dirn == 0;
    // forward: L (primal), U^H (adjoint); backward: U (primal), L^H (adjoint)
    const SweepOperand<R> d0 = sweep_op<R>(fwd ? dinv : dinv + NB * NB, ds, NB, false);
    const SweepOperand<R> d1 = sweep_op<R>(fwd ? dinv + NB * NB : dinv, ds, NB, true);
    const SweepOperand<R> a0 = sweep_op<R>(W, ws, ld, false);
    const SweepOperand<R> a1 = sweep_op<R>(W, ws, ld, true);
    const double tiles = (double)nsteps * (nsteps + 1) / 2.0;  // diagonal + off-diagonal blocks
    trace::Scope ts(st, EXPM_PFD_K_SOLVE_GEMM, 8.0 * nchain * tiles * NB * NB * 16,
                    e * nblk * tiles * NB * NB + 2.0 * e * nchain * npad * 16);
    const unsigned nwg = (unsigned)nchain * (unsigned)nsteps;
    if (nchain >= WHOLE_CHAIN_MIN)
      hipLaunchKernelGGL((k_sweep_whole<R>), dim3((unsigned)nchain), dim3(256), 0, st, fwd ? 1 : 0, nsteps, cpb, d0,
                         d1, a0, a1, PB, X, (int64_t)mp, ldS, gate);
    else
      hipLaunchKernelGGL((k_sweep_chain<R>), dim3(nwg), dim3(256), 0, st, fwd ? 1 : 0, nsteps, nchain, cpb, d0, d1,
                         a0, a1, PB, X, (int64_t)mp, ldS, pl->sweep_sync, gate);
  }
  if (adjoint)
    moves_apply<R>(st, PB, X + (int64_t)PB * mp, mp, ldS, mp, mp, 0, pl->moves, mstride, 0, nsteps, 1, gate);
}

// gate: see KSplit (nullptr: always runs)
template <typename R>
void solves(expm_pfd_plan_t pl, cx<R>* X, int64_t ldS, int mp, bool adjoint, hipStream_t st,
            const int* gate = nullptr) {
  if (mp <= CHAIN_MP_MAX) {
    solves_chain<R>(pl, X, ldS, mp, adjoint, st, gate);
    return;
  }
  const int PB = pl->PB;
  const int npad = (int)pl->npad;
  const int64_t ld = npad, ws = (int64_t)npad * npad;
  const cx<R>* W = (const cx<R>*)pl->W;
  const cx<R>* dinv = (const cx<R>*)pl->dinv;
  const int64_t ds = (int64_t)pl->nsteps * 2 * NB * NB;
  const int64_t mstride = (int64_t)pl->nsteps * MOVE_STRIDE;
  const int nsteps = pl->nsteps;
  const int nb_batch = adjoint ? 2 * PB : PB;  // primal blocks 0..PB-1, adjoint blocks PB..2PB-1
  // P^T on the primal blocks
  moves_apply<R>(st, PB, X, mp, ldS, mp, mp, 0, pl->moves, mstride, 0, nsteps, 0, gate);
  // forward sweeps: L (primal) and U^H (adjoint); diagonal blocks by their inverses
  for (int s = 0; s < nsteps; ++s) {
    const int j0 = s * NB, nb = std::min(NB, npad - j0);
    const int64_t r1 = j0 + nb;
    const int below = npad - j0 - nb;
    const cx<R>* Linv = dinv + (int64_t)s * 2 * NB * NB;
    const cx<R>* Uinv = Linv + NB * NB;
    gemm<R, 1>(st, EXPM_PFD_K_SOLVE_GEMM, nb_batch, nb, mp, nb, opnd<R>(Linv, ds, NB, false),
               opnd<R>(Uinv, ds, NB, true), PB, X + (int64_t)j0 * ldS, mp, ldS, X + (int64_t)j0 * ldS, mp, ldS,
               {1, 0, 0, 0}, 0, gate);
    if (below > 0)
      gemm<R, 0>(st, EXPM_PFD_K_SOLVE_GEMM, nb_batch, below, mp, nb, opnd<R>(W + r1 * ld + j0, ws, ld, false),
                 opnd<R>(W + (int64_t)j0 * ld + r1, ws, ld, true), PB, X + (int64_t)j0 * ldS, mp, ldS, X + r1 * ldS,
                 mp, ldS, {1, 0, 0, 0}, 0, gate);
  }
  // backward sweeps: U (primal) and L^H (adjoint)
  for (int s = nsteps - 1; s >= 0; --s) {
    const int j0 = s * NB, nb = std::min(NB, npad - j0);
    const cx<R>* Linv = dinv + (int64_t)s * 2 * NB * NB;
    const cx<R>* Uinv = Linv + NB * NB;
    gemm<R, 1>(st, EXPM_PFD_K_SOLVE_GEMM, nb_batch, nb, mp, nb, opnd<R>(Uinv, ds, NB, false),
               opnd<R>(Linv, ds, NB, true), PB, X + (int64_t)j0 * ldS, mp, ldS, X + (int64_t)j0 * ldS, mp, ldS,
               {1, 0, 0, 0}, 0, gate);
    if (j0 > 0)
      gemm<R, 0>(st, EXPM_PFD_K_SOLVE_GEMM, nb_batch, j0, mp, nb, opnd<R>(W + j0, ws, ld, false),
                 opnd<R>(W + (int64_t)j0 * ld, ws, ld, true), PB, X + (int64_t)j0 * ldS, mp, ldS, X, mp, ldS,
                 {1, 0, 0, 0}, 0, gate);
  }
  // P on the adjoint blocks
  if (adjoint)
    moves_apply<R>(st, PB, X + (int64_t)PB * mp, mp, ldS, mp, mp, 0, pl->moves, mstride, 0, nsteps, 1, gate);
}

// ---- one pass of the whole path over the plan's G problems ------------------------
// descs: device descriptors (group plans) or nullptr with `one` inline.
// full: V = I for every problem; mp: right-hand-side block width (npad if full);
// nmax, mmax: largest n and m in the group (launch extents).
int run(expm_pfd_plan_t pl, const ProblemDesc* descs, const ProblemDesc& one, bool full, int mp, int nmax, int mmax,
        hipStream_t st) {
  const int P = pl->P, PB = pl->PB, G = pl->G;
  const int npad = (int)pl->npad;
  // adjoint blocks: the conjugate pole's solves (not needed for V = I, where the
  // conjugate term is the adjoint, nor for real data, where it is the conjugate)
  const bool adj = !full && !pl->real_data;
  const int nblk = adj ? 2 * PB : PB;
  const int64_t ldS = (int64_t)nblk * mp;
  const int64_t count = (int64_t)npad * ldS;
  if (ldS > pl->cols_alloc) return EXPM_PFD_ERR_DIM;
  const double e64 = 16.0;
  auto accumulate = [&](const double2* Xsrc) {
    trace::Scope ts(st, EXPM_PFD_K_ACCUM, 8.0 * nblk * (double)nmax * mmax,
                    e64 * ((double)nblk * nmax * mmax + (double)G * nmax * mmax));
    if (full) {
      dim3 g((unsigned)((nmax + 31) / 32), (unsigned)((nmax + 31) / 32), (unsigned)G), b(32, 8);
      hipLaunchKernelGGL(k_accum_full, g, b, 0, st, Xsrc, ldS, npad, P, pl->d_a, descs, one);
    } else {
      dim3 g((unsigned)(((int64_t)nmax * mmax + 255) / 256), (unsigned)G);
      hipLaunchKernelGGL(k_accum_thin, g, dim3(256), 0, st, Xsrc, ldS, mp, PB, P, pl->d_a, descs, one, adj ? 1 : 0);
    }
  };
  if (pl->precision == EXPM_PFD_FP64) {
    factor<double>(pl, descs, one, st);
    double2* Xs = (double2*)pl->Xs;
    {
      trace::Scope ts(st, EXPM_PFD_K_ELEMENTWISE, 0.0, e64 * count);
      hipLaunchKernelGGL((k_stage<double>), dim3(grid_for(count)), dim3(256), 0, st, Xs, ldS, npad, mp, PB, P, descs,
                         one, nullptr);
    }
    solves<double>(pl, Xs, ldS, mp, adj, st);
    accumulate(Xs);
    // per-problem status words (only written where the descriptor names one)
    if (descs) hipLaunchKernelGGL(k_status, dim3((unsigned)G), dim3(256), 0, st, descs, one, nullptr);
    return 0;
  }
  factor<float>(pl, descs, one, st);
  float2* Xs = (float2*)pl->Xs;
  {
    trace::Scope ts(st, EXPM_PFD_K_ELEMENTWISE, 0.0, 8.0 * count);
    hipLaunchKernelGGL((k_stage<float>), dim3(grid_for(count)), dim3(256), 0, st, Xs, ldS, npad, mp, PB, P, descs, one,
                       nullptr);
  }
  solves<float>(pl, Xs, ldS, mp, adj, st);
  {
    trace::Scope ts(st, EXPM_PFD_K_ELEMENTWISE, 0.0, 24.0 * count);
    hipLaunchKernelGGL((k_convert<float, double>), dim3(grid_for(count)), dim3(256), 0, st, Xs, pl->X64, count);
  }
  // Convergence test (ir_tol >= 0): after every sweep, each solve's largest
  // correction against its largest entry.  Once every solve of the launch has
  // converged, the gate word is 0 and the later sweeps' kernels return at once,
  // with no host round trip (captured graphs keep the same launches).
  const bool test = pl->ir_tol >= 0.0;
  int* gate = test ? pl->ir_words : nullptr;
  unsigned* done = test ? (unsigned*)pl->ir_words + 1 : nullptr;
  int* nc = test ? pl->ir_words + 2 : nullptr;
  int* conv = test ? pl->ir_words + 2 + G : nullptr;
  // (with no sweep at all no solve has been shown to meet the tolerance)
  if (test)
    hipLaunchKernelGGL(k_ir_begin, dim3(1), dim3(256), 0, st, gate, nc, G, pl->ir_sweeps == 0 ? 1 : 0, done);
  const int64_t nn = (int64_t)npad * npad;
  // per-block kernels: about 2048 workgroups in all, each block's elements grid-strided
  const int64_t per_blk = (int64_t)npad * mp;
  const dim3 gblk((unsigned)std::max<int64_t>(1, std::min<int64_t>((per_blk + 255) / 256, 2048 / nblk)),
                  (unsigned)nblk);
  for (int it = 0; it < pl->ir_sweeps; ++it) {
    // R = V - (tA + theta I) X in FP64 for every pole solve: one product per
    // problem and half (primal / adjoint blocks) with the problem's FP64 t*A
    {
      trace::Scope ts(st, EXPM_PFD_K_ELEMENTWISE, 0.0, e64 * count);
      hipLaunchKernelGGL((k_stage<double>), dim3(grid_for(count)), dim3(256), 0, st, pl->R64, ldS, npad, mp, PB, P,
                         descs, one, gate);
    }
    if (it >= pl->ir_sweeps - pl->ir_ext) {
      // the last sweeps: residual accumulated in double-double
      trace::Scope ts(st, EXPM_PFD_K_IR_GEMM, 8.0 * (double)npad * npad * ldS,
                      e64 * ((double)G * npad * npad + 3.0 * count) + 8.0 * count);
      hipLaunchKernelGGL(k_residual_dd, dim3((unsigned)(npad / 64), (unsigned)(ldS / 16)), dim3(256), 0, st, pl->Ah,
                         nn, pl->X64, pl->R64, ldS, npad, mp, PB, P, pl->d_theta, descs, one, Xs, gate);
    } else {
      // up to 64 right-hand-side columns per pole: the product in K slices
      // (partials in Rpart, too few output tiles otherwise); wider blocks and
      // V = I: subtracted from R64 directly
      const bool split = !full && mp <= CHAIN_MP_MAX;
      const int S = split ? ir_kslices(npad) : 0;
      const int64_t pstride = (int64_t)npad * ldS;
      if (!split) {
        for (int half = 0; half < (adj ? 2 : 1); ++half) {
          const int64_t off = (int64_t)half * PB * mp;
          gemm<double, 0>(st, EXPM_PFD_K_IR_GEMM, G, npad, P * mp, npad, opnd<double>(pl->Ah, nn, npad, false),
                          opnd<double>(nullptr, 0, 0, false), G, pl->X64 + off, (int64_t)P * mp, ldS, pl->R64 + off,
                          (int64_t)P * mp, ldS, KSplit{1, 0, 0, 0}, 0, gate);
        }
      } else {
        const int Ks = npad / S;
        const KSplit ksp{S, Ks, (int64_t)Ks * ldS, pstride};
        // one launch covers both halves when the group holds one problem
        const int nh = (G == 1 || !adj) ? 1 : 2, ncols = (G == 1 && adj) ? 2 * P * mp : P * mp;
        for (int half = 0; half < nh; ++half) {
          const int64_t off = (int64_t)half * PB * mp;
          gemm<double, 1>(st, EXPM_PFD_K_IR_GEMM, G, npad, ncols, Ks, opnd<double>(pl->Ah, nn, npad, false),
                          opnd<double>(nullptr, 0, 0, false), G, pl->X64 + off, (int64_t)P * mp, ldS,
                          pl->Rpart + off, (int64_t)P * mp, ldS, ksp, 0, gate);
        }
      }
      trace::Scope ts(st, EXPM_PFD_K_ELEMENTWISE, 8.0 * count, (2.0 + S) * e64 * count + 8.0 * count);
      hipLaunchKernelGGL(k_residual32, gblk, dim3(256), 0, st, pl->R64, pl->Rpart, S, pstride, pl->X64, ldS, npad, mp,
                         PB, P, pl->d_theta, descs, one, Xs, gate);
    }
    solves<float>(pl, Xs, ldS, mp, adj, st, gate);
    {
      trace::Scope ts(st, EXPM_PFD_K_ELEMENTWISE, 0.0, 40.0 * count);
      hipLaunchKernelGGL(k_add_correction, gblk, dim3(256), 0, st, pl->X64, Xs, ldS, npad, mp,
                         test ? pl->ir_max : nullptr, gate);
    }
    if (test)
      hipLaunchKernelGGL(k_ir_check, dim3((unsigned)nblk), dim3(64), 0, st, pl->ir_max, nblk, (int)gblk.x, PB, P,
                         pl->ir_tol, gate, nc, conv, done);
  }
  accumulate(pl->X64);
  // per-problem status words (only written where the descriptor names one)
  if (descs) hipLaunchKernelGGL(k_status, dim3((unsigned)G), dim3(256), 0, st, descs, one, nc);
  return 0;
}

int validate_apply(expm_pfd_plan_t pl, const void* A, int64_t lda, const void* V, int64_t ldv, int64_t m, void* X,
                   int64_t ldx) {
  if (!pl || !A || !X) return EXPM_PFD_ERR_NULL;
  if (pl->G != 1) return EXPM_PFD_ERR_ARG;
  if (lda < pl->n || ldx < pl->n) return EXPM_PFD_ERR_LD;
  if (V == nullptr) {
    if (!pl->full_ok || m != pl->n) return EXPM_PFD_ERR_DIM;
  } else {
    if (ldv < pl->n) return EXPM_PFD_ERR_LD;
    const int64_t cap = pl->m_max == 0 ? pl->n : pl->m_max;
    if (m < 1 || m > cap) return EXPM_PFD_ERR_DIM;
  }
  return 0;
}

}  // namespace

extern "C" int expm_pfd_workspace_bytes(int64_t n, int degree, int64_t m_max, const expm_pfd_opts* opts,
                                        size_t* bytes) {
  if (!bytes) return EXPM_PFD_ERR_NULL;
  if (int e = check_degree(degree)) return e;
  if (n < 1 || n > EXPM_PFD_MAX_N || m_max < 0) return EXPM_PFD_ERR_DIM;
  if (int e = check_opts(opts)) return e;
  const bool full_ok = (m_max == 0 || m_max >= n);
  const int64_t mp = round_up(std::min<int64_t>(m_max == 0 ? n : m_max, n), 16);
  *bytes = plan_sizes(round_up(n, NB), 1, degree, mp, full_ok, opts ? opts->precision : EXPM_PFD_FP64).total();
  return 0;
}

extern "C" int expm_pfd_plan(expm_pfd_plan_t* out, int64_t n, int degree, double t, int64_t m_max,
                             const expm_pfd_opts* opts) {
  if (!out) return EXPM_PFD_ERR_NULL;
  *out = nullptr;
  if (int e = check_degree(degree)) return e;
  if (n < 1 || n > EXPM_PFD_MAX_N || m_max < 0) return EXPM_PFD_ERR_DIM;
  if (!std::isfinite(t)) return EXPM_PFD_ERR_ARG;
  if (int e = check_opts(opts)) return e;
  const bool full_ok = (m_max == 0 || m_max >= n);
  const int64_t mp = round_up(std::min<int64_t>(m_max == 0 ? n : m_max, n), 16);
  expm_pfd_plan_t pl = nullptr;
  int rc = create_plan(&pl, round_up(n, NB), 1, degree, mp, full_ok, opts ? opts->precision : EXPM_PFD_FP64, opts);
  if (rc) return rc;
  pl->n = n;
  pl->t = t;
  pl->m_max = m_max;
  pl->upper = opts ? opts->uplo : 0;
  if ((rc = configure_plan(pl, opts)) != 0) {
    free_plan(pl);
    return rc;
  }
  *out = pl;
  return 0;
}

extern "C" int expm_pfd_destroy(expm_pfd_plan_t pl) {
  if (!pl) return EXPM_PFD_ERR_NULL;
  (void)hipDeviceSynchronize();
  free_plan(pl);
  return 0;
}

extern "C" int expm_pfd_apply(expm_pfd_plan_t pl, const void* A, int64_t lda, const void* V, int64_t ldv, int64_t m,
                              void* X, int64_t ldx, void* stream) {
  if (int e = validate_apply(pl, A, lda, V, ldv, m, X, ldx)) return e;
  hipStream_t st = (hipStream_t)stream;
  const bool full = (V == nullptr);
  ProblemDesc one;
  one.A = (const double2*)A;
  one.lda = lda;
  one.V = (const double2*)V;
  one.ldv = ldv;
  one.X = (double2*)X;
  one.ldx = ldx;
  one.t = pl->t;
  one.n = (int)pl->n;
  one.m = (int)m;
  one.real = pl->real_data;
  one.upper = pl->upper;
  one.info = nullptr;
  if (problem_shift(pl->shift, pl->shift_t, pl->t, one)) return EXPM_PFD_ERR_ARG;
  (void)hipGetLastError();
  const int mp = full ? (int)pl->npad : (int)round_up(m, 16);
  if (pl->use_graph && trace::mask == 0) {
    // the graph's kernels read the descriptor from the plan's device copy
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(1), 0, st, pl->d_descs, one);
    const std::pair<int, int64_t> key{full ? 1 : 0, m};
    auto it = pl->graphs.find(key);
    if (it == pl->graphs.end()) {
      hipGraphExec_t ex = nullptr;
      ProblemDesc none{};
      if (int e = capture_graph(
              pl->cap, [&](hipStream_t cs) { return run(pl, pl->d_descs, none, full, mp, (int)pl->n, (int)m, cs); },
              &ex))
        return e;
      it = pl->graphs.emplace(key, ex).first;
    }
    if (hipGraphLaunch(it->second, st) != hipSuccess) return EXPM_PFD_ERR_HIP;
  } else if (int e = run(pl, nullptr, one, full, mp, (int)pl->n, (int)m, st)) {
    return e;
  }
  if (hipGetLastError() != hipSuccess) return EXPM_PFD_ERR_HIP;
  return 0;
}

extern "C" int expm_pfd_plan_check(expm_pfd_plan_t pl) {
  if (!pl) return EXPM_PFD_ERR_NULL;
  if (hipDeviceSynchronize() != hipSuccess) return EXPM_PFD_ERR_HIP;
  const int f = sweep_fault(pl);
  if (f) return f < 0 ? EXPM_PFD_ERR_HIP : EXPM_PFD_ERR_SYNC;
  if (pl->precision == EXPM_PFD_MIXED && pl->ir_tol >= 0.0) {
    int nc = 0;
    if (hipMemcpy(&nc, pl->ir_words + 2, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return EXPM_PFD_ERR_HIP;
    if (nc) return 1;
  }
  return 0;
}

// ============================================================================
// The single-problem path for callers that cannot allocate: the whole plan
// workspace is carved from one fixed device array per GPU.
// ============================================================================
// Host code never hands this name to a kernel or a copy (on the host it only
// stands in for the symbol): the per-device address comes from
// hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[EXPM_PFD_NOALLOC_BYTES];

namespace {

constexpr int SCRATCH_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_at[SCRATCH_DEVICES] = {};  // device address of `scratch` per device (null: not looked up yet)

// The current device's copy of the scratch array (looked up with that device
// current, on its first use).
int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return EXPM_PFD_ERR_HIP;
  if (dev < 0 || dev >= SCRATCH_DEVICES) return EXPM_PFD_ERR_ARG;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_at[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return EXPM_PFD_ERR_HIP;
    }
    scratch_at[dev] = p;
  }
  *out = scratch_at[dev];
  return 0;
}

// Lays the plan's arrays out from `base` (256-byte aligned pieces, in the
// order of plan_sizes) and returns the bytes used; base == nullptr only counts.
size_t carve_plan(expm_pfd_plan_s* pl, const Sizes& sz, char* base, bool mixed) {
  size_t off = 0;
  auto take = [&](auto** p, size_t bytes) {
    if (base) *p = (std::remove_pointer_t<decltype(p)>)(base + off);
    off += round_up((int64_t)bytes, 256);
  };
  take(&pl->d_theta, 64 * sizeof(double2));
  take(&pl->d_a, 64 * sizeof(double2));
  take(&pl->W, sz.w);
  take(&pl->ipiv, sz.ipiv);
  take(&pl->moves, sz.moves);
  take(&pl->dinv, sz.dinv);
  take(&pl->sweep_sync, sz.sweep);
  take(&pl->Xs, sz.xs);
  take(&pl->d_descs, sz.descs);
  if (mixed) {
    take(&pl->Ah, sz.ah);
    take(&pl->X64, sz.x64);
    take(&pl->R64, sz.r64);
    take(&pl->Rpart, sz.rpart);
    take(&pl->ir_words, sz.irw);
    take(&pl->ir_max, sz.irm);
  }
  return off;
}

}  // namespace

extern "C" int expm_pfd_apply_noalloc(int64_t n, int degree, double t, const void* A, int64_t lda, const void* V,
                                      int64_t ldv, int64_t m, void* X, int64_t ldx, const expm_pfd_opts* opts,
                                      int* info, void* stream) {
  if (!A || !X) return EXPM_PFD_ERR_NULL;
  if (int e = check_degree(degree)) return e;
  if (n < 1 || n > EXPM_PFD_MAX_N) return EXPM_PFD_ERR_DIM;
  if (!std::isfinite(t)) return EXPM_PFD_ERR_ARG;
  if (int e = check_opts(opts)) return e;
  if (lda < n || ldx < n) return EXPM_PFD_ERR_LD;
  const bool full = V == nullptr;
  if (full) {
    if (m != n) return EXPM_PFD_ERR_DIM;
  } else {
    if (m < 1 || m > n) return EXPM_PFD_ERR_DIM;
    if (ldv < n) return EXPM_PFD_ERR_LD;
  }
  const int precision = opts ? opts->precision : EXPM_PFD_FP64;
  const bool mixed = precision == EXPM_PFD_MIXED;
  const int64_t npad = round_up(n, NB);
  // the workspace of a plan made for exactly this call (expm_pfd_plan with m_max = m)
  const int64_t mp_max = full ? 16 : round_up(m, 16);
  const Sizes sz = plan_sizes(npad, 1, degree, mp_max, full, precision);
  expm_pfd_plan_s pl;
  if (carve_plan(&pl, sz, nullptr, mixed) > EXPM_PFD_NOALLOC_BYTES) return EXPM_PFD_ERR_SCRATCH;
  init_plan_fields(&pl, npad, 1, degree, mp_max, full, precision, opts ? opts->ir_max_iter : 0,
                   opts ? opts->ir_extended : 0, opts ? opts->real_data : 0, opts ? opts->ir_tol : 0.0);
  ProblemDesc one;
  if (problem_shift(opts ? opts->shift : 0.0, opts ? opts->shift_scale_t : 0, t, one)) return EXPM_PFD_ERR_ARG;
  PoleConsts pc{};
  if (int e = pole_constants(degree, pc.theta, pc.a)) return e;
  void* base = nullptr;
  if (int e = scratch_address(&base)) return e;
  carve_plan(&pl, sz, (char*)base, mixed);
  pl.n = n;
  pl.t = t;
  pl.m_max = full ? 0 : m;
  pl.upper = opts ? opts->uplo : 0;
  pl.lu_tile = opts && opts->lu_tile > 0 ? opts->lu_tile - 1 : 0;
  (void)hipGetDevice(&pl.device);
  hipStream_t st = (hipStream_t)stream;
  (void)hipGetLastError();
  hipLaunchKernelGGL(k_put_consts, dim3(1), dim3(64), 0, st, pl.d_theta, pl.d_a, pc, pl.P);
  // the previous call may have left another layout here: the sweeps' control
  // line and ready flags, and the row moves, start from zero
  hipLaunchKernelGGL(k_fill, dim3(grid_for((int64_t)(sz.sweep / sizeof(int)))), dim3(256), 0, st, pl.sweep_sync,
                     (int64_t)(sz.sweep / sizeof(int)), 0);
  hipLaunchKernelGGL(k_fill, dim3(grid_for((int64_t)(sz.moves / sizeof(int)))), dim3(256), 0, st, pl.moves,
                     (int64_t)(sz.moves / sizeof(int)), 0);
  one.A = (const double2*)A;
  one.lda = lda;
  one.V = (const double2*)V;
  one.ldv = full ? n : ldv;
  one.X = (double2*)X;
  one.ldx = ldx;
  one.t = t;
  one.n = (int)n;
  one.m = (int)m;
  one.real = pl.real_data;
  one.upper = pl.upper;
  one.info = info;
  // the kernels read the descriptor from device memory, as a graph replay does
  hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(1), 0, st, pl.d_descs, one);
  const int mp = full ? (int)npad : (int)round_up(m, 16);
  ProblemDesc none{};
  if (int e = run(&pl, pl.d_descs, none, full, mp, (int)n, (int)m, st)) return e;
  if (info) hipLaunchKernelGGL(k_sweep_status, dim3(1), dim3(64), 0, st, pl.sweep_sync, info, 1, EXPM_PFD_ERR_SYNC);
  return hipGetLastError() == hipSuccess ? 0 : EXPM_PFD_ERR_HIP;
}

// ============================================================================
// batch plans: problems grouped by (padded order, right-hand-side kind), one
// group plan each, all allocated once; every apply uploads the descriptors and
// runs (or replays) the groups without allocating or synchronizing.
// ============================================================================
struct expm_pfd_batch_s {
  struct Group {
    expm_pfd_plan_t pl = nullptr;
    std::vector<int> idx;  // problems of the group, in input order
    bool full = false;
    int mp = 0, nmax = 0, mmax = 0;
    double work = 0;  // G * npad^3: the schedule's load estimate
  };
  int count = 0, degree = 0, real_data = 0, upper = 0, use_graph = 0, autotune = 0, precision = 0;
  double shift = 0.0;  // c of the shifting method (tA units, or A units with shift_t)
  int shift_t = 0;
  int schedule = 0;  // concurrent branches the groups run on (0: not chosen yet)
  std::vector<int64_t> n, m;  // m[i] = 0: V_i = I
  std::vector<Group> groups;
  ProblemDesc* h_descs = nullptr;  // pinned staging of the descriptors, in group order
  hipEvent_t uploaded = nullptr;   // the last upload has read h_descs
  hipStream_t cap = nullptr;       // capture stream
  std::vector<hipStream_t> br;     // branch streams (schedules with more than one branch)
  std::vector<hipEvent_t> ev;      // fork and join events
  std::map<int, hipGraphExec_t> graphs;  // schedule -> executable graph
};

namespace {

constexpr int BATCH_MAX_BRANCHES = 4;

void free_batch(expm_pfd_batch_t b) {
  if (!b) return;
  for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto& g : b->groups) free_plan(g.pl);
  if (b->h_descs) (void)hipHostFree(b->h_descs);
  if (b->uploaded) (void)hipEventDestroy(b->uploaded);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  for (hipStream_t s : b->br) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->ev) (void)hipEventDestroy(e);
  delete b;
}

// Every group's work on `st` (S = 1) or forked over S branch streams, largest
// groups first onto the least loaded branch, joined back into `st`.
int run_groups(expm_pfd_batch_t b, hipStream_t st, int S) {
  ProblemDesc none{};
  S = std::min<int>(S, (int)b->groups.size());
  if (S <= 1) {
    for (auto& g : b->groups)
      if (int e = run(g.pl, g.pl->d_descs, none, g.full, g.mp, g.nmax, g.mmax, st)) return e;
    return 0;
  }
  while ((int)b->br.size() < S) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return EXPM_PFD_ERR_HIP;
    b->br.push_back(s);
  }
  while ((int)b->ev.size() < 1 + S) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return EXPM_PFD_ERR_HIP;
    b->ev.push_back(e);
  }
  if (hipEventRecord(b->ev[0], st) != hipSuccess) return EXPM_PFD_ERR_HIP;
  for (int i = 0; i < S; ++i)
    if (hipStreamWaitEvent(b->br[i], b->ev[0], 0) != hipSuccess) return EXPM_PFD_ERR_HIP;
  std::vector<int> order(b->groups.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return b->groups[x].work > b->groups[y].work; });
  std::vector<double> load(S, 0.0);
  for (int gi : order) {
    auto& g = b->groups[gi];
    const int s = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    load[s] += g.work;
    if (int e = run(g.pl, g.pl->d_descs, none, g.full, g.mp, g.nmax, g.mmax, b->br[s])) return e;
  }
  for (int i = 0; i < S; ++i) {
    if (hipEventRecord(b->ev[1 + i], b->br[i]) != hipSuccess) return EXPM_PFD_ERR_HIP;
    if (hipStreamWaitEvent(st, b->ev[1 + i], 0) != hipSuccess) return EXPM_PFD_ERR_HIP;
  }
  return 0;
}

// One pass over all groups with schedule S: a graph replay, or direct launches
// (no graph requested, or tracing on).
int launch_batch(expm_pfd_batch_t b, hipStream_t st, int S) {
  if (!b->use_graph || trace::mask != 0) return run_groups(b, st, S);
  auto it = b->graphs.find(S);
  if (it == b->graphs.end()) {
    if (!b->cap && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) return EXPM_PFD_ERR_HIP;
    // branch streams and events exist before the capture starts
    if (S > 1) {
      while ((int)b->br.size() < std::min<int>(S, (int)b->groups.size())) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return EXPM_PFD_ERR_HIP;
        b->br.push_back(s);
      }
      while ((int)b->ev.size() < 1 + std::min<int>(S, (int)b->groups.size())) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return EXPM_PFD_ERR_HIP;
        b->ev.push_back(e);
      }
    }
    hipGraphExec_t ex = nullptr;
    if (int e = capture_graph(b->cap, [&](hipStream_t cs) { return run_groups(b, cs, S); }, &ex)) return e;
    it = b->graphs.emplace(S, ex).first;
  }
  return hipGraphLaunch(it->second, st) == hipSuccess ? 0 : EXPM_PFD_ERR_HIP;
}

// First apply: picks the schedule and leaves the batch's result in X.  With
// autotune, each candidate branch count runs the caller's batch once to warm up
// (and capture), then once timed; the fastest is kept.  All candidates compute
// the same bits, so the caller's X is the same whichever ran last.
int choose_schedule(expm_pfd_batch_t b, hipStream_t st) {
  const int G = (int)b->groups.size();
  if (!b->autotune || G == 1) {
    b->schedule = 1;
    return launch_batch(b, st, 1);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  int best = 1, rc = 0;
  float best_ms = 0.f;
  for (int S = 1; S <= std::min(G, BATCH_MAX_BRANCHES) && rc == 0; S *= 2) {
    if ((rc = launch_batch(b, st, S)) != 0) break;
    (void)hipEventRecord(e0, st);
    if ((rc = launch_batch(b, st, S)) != 0) break;
    (void)hipEventRecord(e1, st);
    float ms = 0.f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = EXPM_PFD_ERR_HIP;
      break;
    }
    if (S == 1 || ms < best_ms) {
      best = S;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // keep only the chosen schedule's graph
  for (auto it = b->graphs.begin(); it != b->graphs.end();) {
    if (it->first != best) {
      (void)hipGraphExecDestroy(it->second);
      it = b->graphs.erase(it);
    } else {
      ++it;
    }
  }
  b->schedule = best;
  return rc;
}

}  // namespace

namespace {
int batch_plan_impl(expm_pfd_batch_t* out, int count, const int64_t* n, const int64_t* m, int degree,
                    const expm_pfd_opts* opts, const PoolArg* pool);
}

extern "C" int expm_pfd_batch_plan(expm_pfd_batch_t* out, int count, const int64_t* n, const int64_t* m, int degree,
                                   const expm_pfd_opts* opts) {
  return batch_plan_impl(out, count, n, m, degree, opts, nullptr);
}

namespace {
// pool: as in create_plan (nullptr: hipMalloc; otherwise the stream-ordered pool)
int batch_plan_impl(expm_pfd_batch_t* out, int count, const int64_t* n, const int64_t* m, int degree,
                    const expm_pfd_opts* opts, const PoolArg* pool) {
  if (!out) return EXPM_PFD_ERR_NULL;
  *out = nullptr;
  if (count < 1) return EXPM_PFD_ERR_DIM;
  if (!n || !m) return EXPM_PFD_ERR_NULL;
  if (int e = check_degree(degree)) return e;
  if (int e = check_opts(opts)) return e;
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1 || n[i] > EXPM_PFD_MAX_N) return EXPM_PFD_ERR_DIM;
    if (m[i] < 0 || m[i] > n[i]) return EXPM_PFD_ERR_DIM;
  }
  const int precision = opts ? opts->precision : EXPM_PFD_FP64;
  auto* b = new expm_pfd_batch_s();
  b->count = count;
  b->degree = degree;
  b->real_data = opts ? (opts->real_data ? 1 : 0) : 0;
  b->upper = opts ? opts->uplo : 0;
  b->use_graph = opts ? (opts->graph ? 1 : 0) : 0;
  b->autotune = opts ? (opts->autotune ? 1 : 0) : 0;
  b->precision = precision;
  b->shift = opts ? opts->shift : 0.0;
  b->shift_t = opts && opts->shift_scale_t ? 1 : 0;
  b->n.assign(n, n + count);
  b->m.assign(m, m + count);
  // groups: same padded order and same kind (V = I, or 16-column-rounded width)
  std::map<std::pair<int64_t, int64_t>, std::vector<int>> keyed;
  for (int i = 0; i < count; ++i) keyed[{round_up(n[i], NB), m[i] ? round_up(m[i], 16) : 0}].push_back(i);
  int rc = 0;
  for (auto& kv : keyed) {
    expm_pfd_batch_s::Group g;
    const int64_t npad = kv.first.first, mpk = kv.first.second;
    g.idx = kv.second;
    g.full = mpk == 0;
    g.mp = g.full ? (int)npad : (int)mpk;
    const int G = (int)g.idx.size();
    for (int i : g.idx) {
      g.nmax = std::max<int>(g.nmax, (int)n[i]);
      g.mmax = std::max<int>(g.mmax, (int)(m[i] ? m[i] : n[i]));
    }
    g.work = (double)G * npad * npad * npad;
    rc = create_plan(&g.pl, npad, G, degree, g.full ? 16 : mpk, g.full, precision, opts, pool);
    if (rc) break;
    b->groups.push_back(std::move(g));
    expm_pfd_plan_t pl = b->groups.back().pl;
    if (opts && (opts->lu_tile > 0 || opts->autotune)) {
      expm_pfd_opts o = *opts;
      o.graph = 0;  // graphs are the batch's, not the group plans'
      if ((rc = configure_plan(pl, &o)) != 0) break;
    }
  }
  HipErr he;
  if (!rc) {
    // (the capture stream and the branch streams are created when first needed)
    he(hipHostMalloc((void**)&b->h_descs, (size_t)count * sizeof(ProblemDesc), hipHostMallocDefault));
    he(hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming));
    if (he.e != hipSuccess) rc = he.e == hipErrorOutOfMemory ? EXPM_PFD_ERR_OOM : EXPM_PFD_ERR_HIP;
  }
  if (rc) {
    (void)hipGetLastError();
    free_batch(b);
    return rc;
  }
  *out = b;
  return 0;
}
}  // namespace

extern "C" int expm_pfd_batch_apply(expm_pfd_batch_t b, const double* t, const void* const* A, const int64_t* lda,
                                    const void* const* V, const int64_t* ldv, void* const* X, const int64_t* ldx,
                                    int* info, void* stream) {
  if (!b) return EXPM_PFD_ERR_NULL;
  if (!t || !A || !lda || !V || !ldv || !X || !ldx) return EXPM_PFD_ERR_NULL;
  for (int i = 0; i < b->count; ++i) {
    if (!A[i] || !X[i]) return EXPM_PFD_ERR_NULL;
    if ((V[i] == nullptr) != (b->m[i] == 0)) return EXPM_PFD_ERR_ARG;
    if (lda[i] < b->n[i] || ldx[i] < b->n[i] || (V[i] && ldv[i] < b->n[i])) return EXPM_PFD_ERR_LD;
    if (!std::isfinite(t[i])) return EXPM_PFD_ERR_ARG;
    ProblemDesc d;
    if (problem_shift(b->shift, b->shift_t, t[i], d)) return EXPM_PFD_ERR_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  (void)hipGetLastError();
  // the previous apply's uploads have finished reading the staging buffer
  if (hipEventSynchronize(b->uploaded) != hipSuccess) return EXPM_PFD_ERR_HIP;
  int off = 0;
  for (auto& g : b->groups) {
    ProblemDesc* hd = b->h_descs + off;
    for (size_t k = 0; k < g.idx.size(); ++k) {
      const int i = g.idx[k];
      ProblemDesc& d = hd[k];
      d.A = (const double2*)A[i];
      d.lda = lda[i];
      d.V = (const double2*)V[i];
      d.ldv = V[i] ? ldv[i] : b->n[i];
      d.X = (double2*)X[i];
      d.ldx = ldx[i];
      d.t = t[i];
      d.n = (int)b->n[i];
      d.m = (int)(b->m[i] ? b->m[i] : b->n[i]);
      d.real = b->real_data;
      d.upper = b->upper;
      d.info = info ? info + i : nullptr;
      (void)problem_shift(b->shift, b->shift_t, t[i], d);  // checked above
    }
    if (hipMemcpyAsync(g.pl->d_descs, hd, g.idx.size() * sizeof(ProblemDesc), hipMemcpyHostToDevice, st) !=
        hipSuccess)
      return EXPM_PFD_ERR_HIP;
    off += (int)g.idx.size();
  }
  if (hipEventRecord(b->uploaded, st) != hipSuccess) return EXPM_PFD_ERR_HIP;
  int rc = b->schedule == 0 ? choose_schedule(b, st) : launch_batch(b, st, b->schedule);
  if (!rc && hipGetLastError() != hipSuccess) rc = EXPM_PFD_ERR_HIP;
  return rc;
}

extern "C" int expm_pfd_batch_check(expm_pfd_batch_t b) {
  if (!b) return EXPM_PFD_ERR_NULL;
  if (hipDeviceSynchronize() != hipSuccess) return EXPM_PFD_ERR_HIP;
  for (auto& g : b->groups) {
    const int f = sweep_fault(g.pl);
    if (f < 0) return EXPM_PFD_ERR_HIP;
    if (f) return EXPM_PFD_ERR_SYNC;
  }
  return 0;
}

extern "C" int expm_pfd_batch_info(expm_pfd_batch_t b, int* groups, int* schedule, int* lu_tile_max) {
  if (!b) return EXPM_PFD_ERR_NULL;
  if (groups) *groups = (int)b->groups.size();
  if (schedule) *schedule = b->schedule;
  if (lu_tile_max) {
    int t = 0;
    for (auto& g : b->groups) t = std::max(t, g.pl->lu_tile);
    *lu_tile_max = t;
  }
  return 0;
}

extern "C" int expm_pfd_batch_destroy(expm_pfd_batch_t b) {
  if (!b) return EXPM_PFD_ERR_NULL;
  (void)hipDeviceSynchronize();
  free_batch(b);
  return 0;
}

extern "C" int expm_pfd_apply_batched(int count, const int64_t* n, const double* t, int degree, const void* const* A,
                                      const int64_t* lda, const void* const* V, const int64_t* ldv,
                                      const int64_t* m, void* const* X, const int64_t* ldx,
                                      const expm_pfd_opts* opts, void* stream, int* info) {
  if (count < 1) return EXPM_PFD_ERR_DIM;
  if (!n || !t || !A || !lda || !V || !ldv || !m || !X || !ldx) return EXPM_PFD_ERR_NULL;
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1 || n[i] > EXPM_PFD_MAX_N) return EXPM_PFD_ERR_DIM;
    if (V[i] ? (m[i] < 1 || m[i] > n[i]) : (m[i] != n[i])) return EXPM_PFD_ERR_DIM;
  }
  std::vector<int64_t> mk(count);
  for (int i = 0; i < count; ++i) mk[i] = V[i] ? m[i] : 0;
  // workspace from the stream-ordered pool on the caller's stream: repeated calls
  // reuse it instead of allocating device memory each time
  hipStream_t st = (hipStream_t)stream;
  int dev = 0;
  (void)hipGetDevice(&dev);
  keep_pool_memory(dev);
  const PoolArg pa{st};
  std::vector<int> hinfo(count, 0);
  // one batched pass over the problems listed in `idx`; their status into hinfo
  auto pass = [&](const std::vector<int>& idx, const expm_pfd_opts* o) -> int {
    const int c = (int)idx.size();
    std::vector<int64_t> n2(c), m2(c), lda2(c), ldv2(c), ldx2(c);
    std::vector<double> t2(c);
    std::vector<const void*> A2(c), V2(c);
    std::vector<void*> X2(c);
    for (int k = 0; k < c; ++k) {
      const int i = idx[k];
      n2[k] = n[i], m2[k] = mk[i], lda2[k] = lda[i], ldv2[k] = ldv[i], ldx2[k] = ldx[i], t2[k] = t[i];
      A2[k] = A[i], V2[k] = V[i], X2[k] = X[i];
    }
    expm_pfd_batch_t b = nullptr;
    if (int e = batch_plan_impl(&b, c, n2.data(), m2.data(), degree, o, &pa)) return e;
    int* dinfo = nullptr;
    int rc = 0;
    if (hipMallocAsync((void**)&dinfo, (size_t)c * sizeof(int), st) != hipSuccess) rc = EXPM_PFD_ERR_OOM;
    if (!rc)
      rc = expm_pfd_batch_apply(b, t2.data(), A2.data(), lda2.data(), V2.data(), ldv2.data(), X2.data(), ldx2.data(),
                                dinfo, stream);
    if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = EXPM_PFD_ERR_HIP;
    if (!rc) rc = expm_pfd_batch_check(b);
    std::vector<int> h(c, 0);
    if (!rc && hipMemcpy(h.data(), dinfo, (size_t)c * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
      rc = EXPM_PFD_ERR_HIP;
    for (int k = 0; k < c && !rc; ++k) hinfo[idx[k]] = h[k];
    if (dinfo) (void)hipFreeAsync(dinfo, st);
    expm_pfd_batch_destroy(b);
    return rc;
  };
  std::vector<int> all(count);
  for (int i = 0; i < count; ++i) all[i] = i;
  int rc = pass(all, opts);
  // FP64 fallback: problems whose refinement missed its tolerance are solved
  // again on the FP64 path; their status stays 1 (or 2 for a non-finite result)
  if (!rc && opts && opts->precision == EXPM_PFD_MIXED) {
    std::vector<int> redo;
    for (int i = 0; i < count; ++i)
      if (hinfo[i] == 1) redo.push_back(i);
    if (!redo.empty()) {
      expm_pfd_opts o = *opts;
      o.precision = EXPM_PFD_FP64;
      rc = pass(redo, &o);
      for (int i : redo)
        if (hinfo[i] == 0) hinfo[i] = 1;
    }
  }
  if (!rc && info) std::memcpy(info, hinfo.data(), (size_t)count * sizeof(int));
  return rc;
}

// ============================================================================
// queued serving (continuous batching)
// ============================================================================
struct expm_pfd_queue_s {
  using clock = std::chrono::steady_clock;
  enum { PENDING = 1, DONE = 2, FAIL_BUDGET = 3, FAIL_SYNC = 4, FAIL_HIP = 5 };
  // tridiagonal form of a registered matrix: none yet, wanted (its requests
  // wait for it), being reduced, ready, or not made (no room in the budget)
  enum { TRI_NONE = 0, TRI_WANTED, TRI_REDUCING, TRI_READY, TRI_SKIP };
  enum { FLIGHT_LU = 0, FLIGHT_REDUCE, FLIGHT_TRI };
  struct Req {
    uint64_t ticket = 0;
    int64_t mat = -1;                // registered matrix, or -1: the caller's A read in place
    const double2* A = nullptr;      // the matrix the request reads
    int64_t n = 0, lda = 0;
    double t = 1.0;
    const void* V = nullptr;
    int64_t m = 0, ldv = 0;
    void* X = nullptr;
    int64_t ldx = 0;
    hipEvent_t ready = nullptr;      // recorded on the caller's stream at submit (inputs written)
    hipEvent_t mat_ready = nullptr;  // the registered copy is complete
    clock::time_point submitted;
    int fp64 = 0;                    // FP64 re-solve after the mixed refinement missed its tolerance
  };
  struct Mat {
    double2* A = nullptr;
    int64_t n = 0;
    size_t bytes = 0;
    int refs = 0;           // requests submitted and not yet completed, and a reduction in flight
    bool released = false;  // unregistered: freed once refs is 0
    hipEvent_t ready = nullptr;
    int64_t uses = 0;             // requests submitted for it
    int tri_state = TRI_NONE;
    expm_pfd_tri_t tri = nullptr;  // its tridiagonal form, once reduced
    size_t tri_bytes = 0;          // device bytes of `tri` (counted with the matrices)
    bool tri_busy = false;         // a flight of tridiagonal applies on it is in progress
  };
  struct Flight {
    int kind = FLIGHT_LU;
    int64_t mat = -1;              // FLIGHT_REDUCE, FLIGHT_TRI: the registered matrix
    expm_pfd_tri_t tri = nullptr;  // ... and its tridiagonal plan
    std::vector<int> rc;           // FLIGHT_TRI: launch status of each request's apply
    std::vector<Req> reqs;
    std::vector<ProblemDesc> descs;  // source of the descriptor upload, kept until completion
    expm_pfd_plan_t plan = nullptr;
    size_t bytes = 0;
    bool launched = false;  // its work is enqueued and its stream event recorded
  };
  struct Ticket {
    int state = PENDING;
    int info = 0;
  };

  std::mutex mu;
  std::condition_variable cv;         // scheduler: new requests, completed flights, freed memory, stop
  std::condition_variable cv_flight;  // waiters: a flight was launched on their stream
  std::condition_variable cv_done;    // callers: a ticket completed
  std::deque<Req> pending;
  std::unordered_map<uint64_t, Ticket> tickets;
  std::map<int64_t, Mat> mats;
  int64_t next_mat = 0;
  std::deque<int64_t> want_tri;  // matrices whose reduction is to be launched, in order
  std::vector<std::unique_ptr<Flight>> flight;  // per worker stream: the flight in progress (or null)
  std::map<std::tuple<int64_t, int, int>, std::vector<expm_pfd_plan_t>> free_plans;  // (npad, Gcap, precision)
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> stream_ev;  // per worker stream: completion of its flight (blocking sync)
  hipStream_t aux = nullptr;          // frees of released matrices
  int* dev_status = nullptr;          // per worker stream: max_group status words on the device ...
  int* host_status = nullptr;         // ... and their pinned host copies
  std::vector<hipEvent_t> event_pool;
  std::thread worker;
  std::vector<std::thread> waiters;
  bool stop = false;          // no more submissions: the scheduler ends once all is done
  bool stop_waiters = false;  // set after the scheduler has ended
  size_t budget = 0, mat_bytes = 0, flight_bytes = 0, cached_bytes = 0, peak = 0;
  expm_pfd_opts opts{};  // precision and refinement options of every request
  int degree = 16, max_group = 64, device = 0;
  uint64_t next_ticket = 1;
  int64_t submitted = 0, completed = 0, failed = 0, fallbacks = 0, groups = 0, grouped = 0, padded_up = 0;
  int64_t tri_requests = 0, reductions = 0;
  std::vector<double> lat_ms;
  clock::time_point first_submit, last_done;
  bool any_submit = false;

  // Orders within one group: the padded order of the group is the largest of
  // its requests; a request joins when the group's orders stay within a factor
  // 2 of each other in LU work (hi^3 <= 2 lo^3), or when every order is at
  // most SMALL_PAD, where a pass is bound by its launch sequence rather than
  // by its arithmetic.
  static constexpr int64_t SMALL_PAD = 256;
  static bool orders_compatible(int64_t lo, int64_t hi) { return hi <= SMALL_PAD || hi * hi * hi <= 2 * lo * lo * lo; }

  size_t plan_bytes(int64_t npad, int Gcap, int prec) const {
    return plan_sizes(npad, Gcap, degree, 16, false, prec).total();
  }
  static int capacity_for(int G) {  // plans are cached by capacity: powers of two
    int c = 1;
    while (c < G) c <<= 1;
    return c;
  }
  size_t held() const { return mat_bytes + flight_bytes + cached_bytes; }
  void note_peak() { peak = std::max(peak, held()); }
  hipEvent_t take_event() {
    if (!event_pool.empty()) {
      hipEvent_t e = event_pool.back();
      event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
    return e;
  }
  void give_event(hipEvent_t e) {
    if (e) event_pool.push_back(e);
  }
  // free cached plans until `need` more bytes fit the budget
  void release_cached(size_t need) {
    for (auto it = free_plans.begin(); it != free_plans.end() && held() + need > budget;) {
      auto& v = it->second;
      while (!v.empty() && held() + need > budget) {
        cached_bytes -= plan_bytes(std::get<0>(it->first), std::get<1>(it->first), std::get<2>(it->first));
        free_plan(v.back());
        v.pop_back();
      }
      it = v.empty() ? free_plans.erase(it) : std::next(it);
    }
  }
  void free_matrix(std::map<int64_t, Mat>::iterator it) {
    Mat& mt = it->second;
    // the copy may still be in flight on the registering stream
    (void)hipStreamWaitEvent(aux, mt.ready, 0);
    (void)hipFreeAsync(mt.A, aux);
    // every reduction and apply on the tridiagonal plan has completed (refs is 0)
    if (mt.tri) tri_release(mt.tri, aux);
    give_event(mt.ready);
    mat_bytes -= mt.bytes + mt.tri_bytes;
    mats.erase(it);
  }
  void drop_ref(int64_t mat) {
    if (mat < 0) return;
    auto it = mats.find(mat);
    if (it == mats.end()) return;
    if (--it->second.refs == 0 && it->second.released) free_matrix(it);
  }
  // columns a tridiagonal plan of order n is made for (the requests' limit)
  static int64_t tri_columns(int64_t n) { return std::min<int64_t>(16, n); }
  // the request waits for, or is served on, its matrix's tridiagonal form
  bool tri_routed(const Req& r) const {
    if (r.mat < 0) return false;
    auto it = mats.find(r.mat);
    if (it == mats.end()) return false;
    const int st = it->second.tri_state;
    return (st == TRI_WANTED || st == TRI_REDUCING || st == TRI_READY) && r.m <= tri_columns(r.n);
  }
  void finish(Req& r, int state, int info, clock::time_point now) {
    Ticket& tk = tickets[r.ticket];
    tk.state = state;
    tk.info = info;
    if (state == DONE) {
      lat_ms.push_back(std::chrono::duration<double, std::milli>(now - r.submitted).count());
      ++completed;
      last_done = now;
    } else {
      ++failed;
    }
    give_event(r.ready);
    r.ready = nullptr;
    drop_ref(r.mat);
  }
  // Completion of stream s's flight (its event has completed): statuses from the
  // pinned copies, FP64 re-solves queued for requests whose refinement missed
  // its tolerance, the plan back to the cache.
  void retire(int s) {
    Flight& f = *flight[s];
    const auto now = clock::now();
    if (f.kind != FLIGHT_LU) {
      if (f.kind == FLIGHT_REDUCE) {
        Mat& mt = mats[f.mat];
        mt.tri = f.tri;
        mt.tri_state = TRI_READY;
        ++reductions;
        drop_ref(f.mat);
      } else {
        mats[f.mat].tri_busy = false;  // (before the last request may free the matrix)
        for (size_t k = 0; k < f.reqs.size(); ++k) finish(f.reqs[k], f.rc[k] ? FAIL_HIP : DONE, 0, now);
      }
      flight[s].reset();
      cv_done.notify_all();
      cv.notify_all();
      return;
    }
    const int* st = host_status + (size_t)s * max_group;
    bool sync_fault = false;
    std::vector<Req> redo;
    for (size_t k = 0; k < f.reqs.size(); ++k) {
      Req& r = f.reqs[k];
      const int code = st[k];
      if (code == EXPM_PFD_ERR_SYNC) {
        sync_fault = true;
        finish(r, FAIL_SYNC, 0, now);
      } else if (code == 1 && !r.fp64) {
        Req again = r;
        again.fp64 = 1;
        redo.push_back(again);
      } else {
        // a re-solve on the FP64 path keeps status 1 (2 if its result is not finite)
        finish(r, DONE, r.fp64 && code == 0 ? 1 : code, now);
      }
    }
    // re-solves go first, oldest first (their inputs are still the caller's)
    for (auto it = redo.rbegin(); it != redo.rend(); ++it) pending.push_front(*it);
    fallbacks += (int64_t)redo.size();
    flight_bytes -= f.bytes;
    if (sync_fault) {
      free_plan(f.plan);  // its sweep control line can no longer be trusted
    } else {
      cached_bytes += f.bytes;
      free_plans[std::make_tuple(f.plan->npad, f.plan->Gcap, f.plan->precision)].push_back(f.plan);
    }
    flight[s].reset();
    cv_done.notify_all();
    cv.notify_all();
  }
  // Launch one group on a free stream; false if nothing could be launched.
  // Called with `lk` held; the group is chosen under the lock, its launches are
  // enqueued with the lock released (a group is hundreds of launches, which
  // submitters and the waiters should not wait for).
  bool launch_one(std::unique_lock<std::mutex>& lk) {
    int s = -1;
    for (int i = 0; i < (int)streams.size(); ++i)
      if (!flight[i]) {
        s = i;
        break;
      }
    if (s < 0) return false;
    if (!want_tri.empty()) return launch_reduction(lk, s);
    if (launch_tri(lk, s)) return true;
    // the oldest request on the LU route
    size_t i0 = 0;
    while (i0 < pending.size() && tri_routed(pending[i0])) ++i0;
    if (i0 == pending.size()) return false;
    const int prec = pending[i0].fp64 ? EXPM_PFD_FP64 : opts.precision;
    // the group: the oldest request, then later ones (same precision) in arrival
    // order while the orders stay compatible
    std::vector<size_t> pick;
    int64_t lo = round_up(pending[i0].n, NB), hi = lo;
    for (size_t i = i0; i < pending.size() && (int)pick.size() < max_group; ++i) {
      const Req& r = pending[i];
      if ((r.fp64 ? EXPM_PFD_FP64 : opts.precision) != prec || tri_routed(r)) continue;
      const int64_t np = round_up(r.n, NB);
      const int64_t nlo = std::min(lo, np), nhi = std::max(hi, np);
      if (!orders_compatible(nlo, nhi)) continue;
      lo = nlo;
      hi = nhi;
      pick.push_back(i);
    }
    // largest leading part of the group whose workspace fits next to the
    // registered matrices and the flights (idle cached plans can be released)
    int G = (int)pick.size(), Gcap = capacity_for(G);
    auto reusable = [&](int cap) {
      auto it = free_plans.find(std::make_tuple(hi, cap, prec));
      return it != free_plans.end() && !it->second.empty();
    };
    // a group's workspace stays within a quarter of the budget, so that several
    // flights run side by side (large orders gain nothing from wider groups: their
    // LU is bound by its arithmetic)
    while (Gcap > 1 && plan_bytes(hi, Gcap, prec) > budget / 4) {
      Gcap /= 2;
      G = std::min(G, Gcap);
    }
    for (;;) {
      if (reusable(Gcap) || mat_bytes + flight_bytes + plan_bytes(hi, Gcap, prec) <= budget) break;
      if (Gcap == 1) return false;
      Gcap /= 2;
      G = std::min(G, Gcap);
    }
    pick.resize(G);
    int64_t npad = 0;  // the group's order after trimming
    for (size_t i : pick) npad = std::max(npad, round_up(pending[i].n, NB));
    expm_pfd_plan_t pl = nullptr;
    const size_t bytes = plan_bytes(npad, Gcap, prec);
    auto it = free_plans.find(std::make_tuple(npad, Gcap, prec));
    if (it != free_plans.end() && !it->second.empty()) {
      pl = it->second.back();
      it->second.pop_back();
      cached_bytes -= bytes;
    } else {
      release_cached(bytes);
      if (mat_bytes + flight_bytes + bytes > budget) return false;
    }
    auto f = std::make_unique<Flight>();
    f->plan = pl;
    f->bytes = bytes;
    for (int g = G - 1; g >= 0; --g) {  // erase from the back so earlier indices stay valid
      f->reqs.push_back(pending[pick[g]]);
      pending.erase(pending.begin() + (int64_t)pick[g]);
    }
    std::reverse(f->reqs.begin(), f->reqs.end());
    int nmax = 0, mmax = 0;
    int* dst = dev_status + (size_t)s * max_group;
    for (size_t k = 0; k < f->reqs.size(); ++k) {
      const Req& r = f->reqs[k];
      ProblemDesc d;
      d.A = r.A;
      d.lda = r.lda;
      d.V = (const double2*)r.V;
      d.ldv = r.ldv;
      d.X = (double2*)r.X;
      d.ldx = r.ldx;
      d.t = r.t;
      d.n = (int)r.n;
      d.m = (int)r.m;
      d.real = opts.real_data ? 1 : 0;
      d.upper = opts.uplo;
      d.info = dst + k;
      (void)problem_shift(opts.shift, opts.shift_scale_t, r.t, d);  // checked at submit
      nmax = std::max(nmax, d.n);
      mmax = std::max(mmax, d.m);
      if (round_up(r.n, NB) < npad) ++padded_up;
      f->descs.push_back(d);
    }
    flight_bytes += bytes;
    note_peak();
    ++groups;
    grouped += G;
    Flight* fl = f.get();
    flight[s] = std::move(f);  // the stream is taken; its waiter sleeps until `launched`
    lk.unlock();
    // ---- enqueue without the lock ----
    hipStream_t st = streams[s];
    bool ok = true;
    if (!pl) {
      const PoolArg pa{st};
      expm_pfd_opts o = opts;
      o.precision = prec;
      ok = create_plan(&pl, npad, Gcap, degree, 16, false, prec, &o, &pa) == 0;
      if (!ok) {
        // the device is short although the budget is not: release the idle cached
        // plans, hand the pool's unused memory back and try once more
        (void)hipGetLastError();
        lk.lock();
        release_cached((size_t)-1 / 2);
        lk.unlock();
        (void)hipDeviceSynchronize();  // the released plans' frees are ordered on their own streams
        hipMemPool_t mpool = nullptr;
        if (hipDeviceGetDefaultMemPool(&mpool, device) == hipSuccess) (void)hipMemPoolTrimTo(mpool, 0);
        ok = create_plan(&pl, npad, Gcap, degree, 16, false, prec, &o, &pa) == 0;
      }
      if (ok) pl->lu_tile = opts.lu_tile > 0 ? opts.lu_tile - 1 : 0;
    }
    if (ok) {
      for (const Req& r : fl->reqs) {
        if (r.ready) (void)hipStreamWaitEvent(st, r.ready, 0);
        if (r.mat_ready) (void)hipStreamWaitEvent(st, r.mat_ready, 0);
      }
      pl->G = G;
      pl->PB = G * pl->P;
      (void)hipMemcpyAsync(pl->d_descs, fl->descs.data(), G * sizeof(ProblemDesc), hipMemcpyHostToDevice, st);
      ProblemDesc none{};
      (void)run(pl, pl->d_descs, none, false, 16, nmax, mmax, st);
      hipLaunchKernelGGL(k_sweep_status, dim3(1), dim3(64), 0, st, pl->sweep_sync, dst, G, EXPM_PFD_ERR_SYNC);
      (void)hipMemcpyAsync(host_status + (size_t)s * max_group, dst, G * sizeof(int), hipMemcpyDeviceToHost, st);
      (void)hipEventRecord(stream_ev[s], st);
    } else {
      (void)hipGetLastError();
    }
    lk.lock();
    if (!ok) {
      // no workspace after all: the requests go back to the front, oldest first
      for (auto r = fl->reqs.rbegin(); r != fl->reqs.rend(); ++r) pending.push_front(*r);
      flight_bytes -= bytes;
      --groups;
      grouped -= G;
      flight[s].reset();
      return false;
    }
    fl->plan = pl;
    fl->launched = true;
    cv_flight.notify_all();
    return true;
  }
  // Reduction of the oldest wanted matrix to tridiagonal form on stream s; its
  // plan memory is counted with the matrices. Without room in the budget the
  // matrix keeps the LU route. True: the queue's state changed.
  bool launch_reduction(std::unique_lock<std::mutex>& lk, int s) {
    const int64_t id = want_tri.front();
    want_tri.pop_front();
    auto it = mats.find(id);
    if (it == mats.end()) return true;
    Mat& mt = it->second;
    if (mt.released) {
      mt.tri_state = TRI_SKIP;
      return true;
    }
    const int64_t cols = tri_columns(mt.n);
    const size_t bytes = tri_bytes(mt.n, degree, cols);
    release_cached(bytes);
    if (mat_bytes + flight_bytes + bytes > budget) {
      mt.tri_state = TRI_SKIP;
      return true;
    }
    mt.tri_state = TRI_REDUCING;
    mt.tri_bytes = bytes;
    mat_bytes += bytes;
    ++mt.refs;
    note_peak();
    auto f = std::make_unique<Flight>();
    f->kind = FLIGHT_REDUCE;
    f->mat = id;
    Flight* fl = f.get();
    flight[s] = std::move(f);
    const double2* A = mt.A;
    const int64_t n = mt.n;
    hipEvent_t mat_ready = mt.ready;
    lk.unlock();
    // ---- enqueue without the lock ----
    hipStream_t st = streams[s];
    expm_pfd_tri_t tri = nullptr;
    bool ok = tri_create(&tri, n, degree, cols, &opts, st) == 0;
    ok = ok && hipStreamWaitEvent(st, mat_ready, 0) == hipSuccess;
    ok = ok && expm_pfd_tridiag_factor(tri, A, n, st) == 0;
    ok = ok && hipEventRecord(stream_ev[s], st) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      if (tri) {
        (void)hipStreamSynchronize(st);
        tri_release(tri, st);
      }
    }
    lk.lock();
    if (!ok) {
      Mat& m2 = mats[id];
      m2.tri_state = TRI_SKIP;
      mat_bytes -= m2.tri_bytes;
      m2.tri_bytes = 0;
      flight[s].reset();
      drop_ref(id);
      return true;
    }
    fl->tri = tri;
    fl->launched = true;
    cv_flight.notify_all();
    return true;
  }
  // The waiting requests of one reduced matrix (oldest first, up to max_group)
  // applied one after another on stream s; one such flight per matrix at a time,
  // as the applies share the plan's buffers. False: none to launch.
  bool launch_tri(std::unique_lock<std::mutex>& lk, int s) {
    int64_t id = -1;
    std::vector<size_t> pick;
    for (size_t i = 0; i < pending.size() && (int)pick.size() < max_group; ++i) {
      const Req& r = pending[i];
      if (!tri_routed(r)) continue;
      const Mat& mt = mats.find(r.mat)->second;
      if (mt.tri_state != TRI_READY || mt.tri_busy) continue;
      if (id < 0) id = r.mat;
      if (r.mat == id) pick.push_back(i);
    }
    if (pick.empty()) return false;
    Mat& mt = mats[id];
    mt.tri_busy = true;
    auto f = std::make_unique<Flight>();
    f->kind = FLIGHT_TRI;
    f->mat = id;
    f->tri = mt.tri;
    for (auto g = pick.rbegin(); g != pick.rend(); ++g) {
      f->reqs.push_back(pending[*g]);
      pending.erase(pending.begin() + (int64_t)*g);
    }
    std::reverse(f->reqs.begin(), f->reqs.end());
    f->rc.assign(f->reqs.size(), 0);
    tri_requests += (int64_t)f->reqs.size();
    Flight* fl = f.get();
    flight[s] = std::move(f);
    lk.unlock();
    // ---- enqueue without the lock ----
    hipStream_t st = streams[s];
    for (size_t k = 0; k < fl->reqs.size(); ++k) {
      const Req& r = fl->reqs[k];
      if (r.ready) (void)hipStreamWaitEvent(st, r.ready, 0);
      fl->rc[k] = expm_pfd_tridiag_apply(fl->tri, r.t, r.V, r.ldv, r.m, r.X, r.ldx, st);
    }
    (void)hipEventRecord(stream_ev[s], st);
    lk.lock();
    fl->launched = true;
    cv_flight.notify_all();
    return true;
  }
  void loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      while (launch_one(lk)) {
      }
      bool any_flight = false;
      for (auto& f : flight) any_flight |= (bool)f;
      if (!any_flight && !pending.empty()) {
        // nothing runs and the oldest request still does not fit (matrices were
        // registered after it was submitted): fail it rather than wait forever
        Req r = pending.front();
        pending.pop_front();
        finish(r, FAIL_BUDGET, 0, clock::now());
        cv_done.notify_all();
        continue;
      }
      if (stop && pending.empty() && !any_flight) break;
      cv.wait(lk);
    }
  }
  // One thread per worker stream: sleeps on the stream's flight event and
  // retires the flight when it completes.
  void wait_loop(int s) {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv_flight.wait(lk, [&] { return stop_waiters || (flight[s] && flight[s]->launched); });
      if (!flight[s]) break;  // the scheduler has ended and nothing is in flight here
      hipEvent_t ev = stream_ev[s];
      lk.unlock();
      (void)hipEventSynchronize(ev);
      lk.lock();
      retire(s);
    }
  }
};

extern "C" int expm_pfd_queue_create(expm_pfd_queue_t* out, size_t hbm_budget, int degree, const expm_pfd_opts* opts,
                                     int max_group, int nstreams) {
  if (!out) return EXPM_PFD_ERR_NULL;
  *out = nullptr;
  if (int e = check_degree(degree)) return e;
  if (int e = check_opts(opts)) return e;
  // the tridiagonal route reads imaginary parts: not with real_data
  if (opts && opts->tridiag_reuse > 0 && opts->real_data) return EXPM_PFD_ERR_ARG;
  auto* q = new expm_pfd_queue_s();
  q->budget = hbm_budget;
  q->degree = degree;
  if (opts) q->opts = *opts;
  q->opts.graph = 0;
  q->opts.autotune = 0;
  q->max_group = max_group > 0 ? max_group : 64;
  (void)hipGetDevice(&q->device);
  const int ns = nstreams > 0 ? nstreams : 3;
  HipErr he;
  for (int i = 0; i < ns && he.e == hipSuccess; ++i) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    he(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    he(hipEventCreateWithFlags(&ev, hipEventDisableTiming | hipEventBlockingSync));
    q->streams.push_back(st);
    q->stream_ev.push_back(ev);
    q->flight.emplace_back();
  }
  he(hipStreamCreateWithFlags(&q->aux, hipStreamNonBlocking));
  he(hipMalloc((void**)&q->dev_status, (size_t)ns * q->max_group * sizeof(int)));
  he(hipHostMalloc((void**)&q->host_status, (size_t)ns * q->max_group * sizeof(int), hipHostMallocDefault));
  if (he.e != hipSuccess) {
    (void)hipGetLastError();
    for (hipStream_t x : q->streams)
      if (x) (void)hipStreamDestroy(x);
    for (hipEvent_t e : q->stream_ev)
      if (e) (void)hipEventDestroy(e);
    if (q->aux) (void)hipStreamDestroy(q->aux);
    if (q->dev_status) (void)hipFree(q->dev_status);
    if (q->host_status) (void)hipHostFree(q->host_status);
    delete q;
    return he.e == hipErrorOutOfMemory ? EXPM_PFD_ERR_OOM : EXPM_PFD_ERR_HIP;
  }
  // freed plan workspace stays in the device's stream-ordered pool, so plans of
  // new shapes are carved from it without new device allocations
  keep_pool_memory(q->device);
  q->worker = std::thread([q] { q->loop(); });
  for (int i = 0; i < ns; ++i) q->waiters.emplace_back([q, i] { q->wait_loop(i); });
  *out = q;
  return 0;
}

extern "C" int expm_pfd_register_matrix(expm_pfd_queue_t q, const void* A, int64_t n, int64_t lda, void* stream,
                                        int64_t* mat_id) {
  if (!q || !A || !mat_id) return EXPM_PFD_ERR_NULL;
  if (n < 1 || n > EXPM_PFD_MAX_N) return EXPM_PFD_ERR_DIM;
  if (lda < n) return EXPM_PFD_ERR_LD;
  const size_t bytes = (size_t)n * n * sizeof(double2);
  hipStream_t st = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(q->mu);
  q->release_cached(bytes);
  if (q->mat_bytes + q->flight_bytes + bytes > q->budget) return EXPM_PFD_ERR_BUDGET;
  double2* d = nullptr;
  hipEvent_t ev = q->take_event();
  // stream-ordered: the copy follows the caller's work that wrote A; requests
  // wait for `ev` before they read the copy
  bool got = ev && hipMallocAsync((void**)&d, bytes, st) == hipSuccess;
  if (!got && ev) {
    // the device is short although the budget is not (the pool's free blocks do
    // not fit this size): release the idle cached plans, hand the pool's unused
    // memory back and try once more
    (void)hipGetLastError();
    q->release_cached((size_t)-1 / 2);
    (void)hipDeviceSynchronize();
    hipMemPool_t mpool = nullptr;
    if (hipDeviceGetDefaultMemPool(&mpool, q->device) == hipSuccess) (void)hipMemPoolTrimTo(mpool, 0);
    got = hipMallocAsync((void**)&d, bytes, st) == hipSuccess;
  }
  if (!got) {
    (void)hipGetLastError();
    q->give_event(ev);
    return EXPM_PFD_ERR_OOM;
  }
  if (hipMemcpy2DAsync(d, n * sizeof(double2), A, lda * sizeof(double2), n * sizeof(double2), n,
                       hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipEventRecord(ev, st) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFreeAsync(d, st);
    q->give_event(ev);
    return EXPM_PFD_ERR_HIP;
  }
  expm_pfd_queue_s::Mat m;
  m.A = d;
  m.n = n;
  m.bytes = bytes;
  m.ready = ev;
  const int64_t id = q->next_mat++;
  q->mats.emplace(id, m);
  q->mat_bytes += bytes;
  q->note_peak();
  *mat_id = id;
  return 0;
}

extern "C" int expm_pfd_unregister_matrix(expm_pfd_queue_t q, int64_t mat_id) {
  if (!q) return EXPM_PFD_ERR_NULL;
  std::lock_guard<std::mutex> lk(q->mu);
  auto it = q->mats.find(mat_id);
  if (it == q->mats.end() || it->second.released) return EXPM_PFD_ERR_TICKET;
  it->second.released = true;
  if (it->second.refs == 0) q->free_matrix(it);
  q->cv.notify_all();
  return 0;
}

extern "C" int expm_pfd_submit(expm_pfd_queue_t q, int64_t mat_id, const void* A, int64_t n, int64_t lda, double t,
                               const void* V, int64_t m, int64_t ldv, void* X, int64_t ldx, void* stream,
                               uint64_t* ticket) {
  if (!q || !V || !X || !ticket) return EXPM_PFD_ERR_NULL;
  if (!std::isfinite(t)) return EXPM_PFD_ERR_ARG;
  ProblemDesc probe;
  if (problem_shift(q->opts.shift, q->opts.shift_scale_t, t, probe)) return EXPM_PFD_ERR_ARG;
  std::lock_guard<std::mutex> lk(q->mu);
  expm_pfd_queue_s::Req r;
  if (A == nullptr) {
    auto it = q->mats.find(mat_id);
    if (it == q->mats.end() || it->second.released) return EXPM_PFD_ERR_TICKET;
    r.mat = mat_id;
    r.A = it->second.A;
    r.n = it->second.n;
    r.lda = it->second.n;
    r.mat_ready = it->second.ready;
  } else {
    if (n < 1 || n > EXPM_PFD_MAX_N) return EXPM_PFD_ERR_DIM;
    if (lda < n) return EXPM_PFD_ERR_LD;
    r.A = (const double2*)A;
    r.n = n;
    r.lda = lda;
  }
  if (m < 1 || m > 16) return EXPM_PFD_ERR_DIM;
  if (ldv < r.n || ldx < r.n) return EXPM_PFD_ERR_LD;
  if (q->mat_bytes + q->plan_bytes(round_up(r.n, NB), 1, q->opts.precision) > q->budget) return EXPM_PFD_ERR_BUDGET;
  r.ready = q->take_event();
  if (!r.ready || hipEventRecord(r.ready, (hipStream_t)stream) != hipSuccess) {
    (void)hipGetLastError();
    q->give_event(r.ready);
    return EXPM_PFD_ERR_HIP;
  }
  if (r.mat >= 0) {
    expm_pfd_queue_s::Mat& mt = q->mats[r.mat];
    ++mt.refs;
    // the request that brings a matrix to its reuse threshold asks for its
    // reduction; it and the later requests wait for the tridiagonal form
    if (q->opts.tridiag_reuse > 0 && ++mt.uses >= q->opts.tridiag_reuse && mt.tri_state == expm_pfd_queue_s::TRI_NONE) {
      mt.tri_state = expm_pfd_queue_s::TRI_WANTED;
      q->want_tri.push_back(r.mat);
    }
  }
  r.ticket = q->next_ticket++;
  r.t = t;
  r.V = V;
  r.m = m;
  r.ldv = ldv;
  r.X = X;
  r.ldx = ldx;
  r.submitted = expm_pfd_queue_s::clock::now();
  if (!q->any_submit) {
    q->first_submit = r.submitted;
    q->any_submit = true;
  }
  q->pending.push_back(r);
  q->tickets[r.ticket] = expm_pfd_queue_s::Ticket{};
  ++q->submitted;
  *ticket = r.ticket;
  q->cv.notify_all();
  return 0;
}

static int state_error(int st) {
  return st == expm_pfd_queue_s::FAIL_BUDGET ? EXPM_PFD_ERR_BUDGET
         : st == expm_pfd_queue_s::FAIL_SYNC ? EXPM_PFD_ERR_SYNC
         : st == expm_pfd_queue_s::FAIL_HIP  ? EXPM_PFD_ERR_HIP
                                              : 0;
}

extern "C" int expm_pfd_poll(expm_pfd_queue_t q, uint64_t ticket, int* done, int* info) {
  if (!q || !done) return EXPM_PFD_ERR_NULL;
  std::lock_guard<std::mutex> lk(q->mu);
  auto it = q->tickets.find(ticket);
  if (it == q->tickets.end()) return EXPM_PFD_ERR_TICKET;
  *done = it->second.state == expm_pfd_queue_s::DONE ? 1 : 0;
  if (info) *info = it->second.info;
  return state_error(it->second.state);
}

extern "C" int expm_pfd_wait(expm_pfd_queue_t q, uint64_t ticket, int* info) {
  if (!q) return EXPM_PFD_ERR_NULL;
  std::unique_lock<std::mutex> lk(q->mu);
  if (q->tickets.find(ticket) == q->tickets.end()) return EXPM_PFD_ERR_TICKET;
  // (a lookup each time: submissions may rehash the table while this waits)
  q->cv_done.wait(lk, [&] { return q->tickets[ticket].state != expm_pfd_queue_s::PENDING; });
  const expm_pfd_queue_s::Ticket tk = q->tickets[ticket];
  if (info) *info = tk.info;
  return state_error(tk.state);
}

extern "C" int expm_pfd_queue_drain(expm_pfd_queue_t q) {
  if (!q) return EXPM_PFD_ERR_NULL;
  std::unique_lock<std::mutex> lk(q->mu);
  q->cv_done.wait(lk, [&] { return q->completed + q->failed == q->submitted; });
  if (q->failed == 0) return 0;
  // the first failure kind found among the tickets
  for (auto& kv : q->tickets)
    if (int e = state_error(kv.second.state)) return e;
  return EXPM_PFD_ERR_HIP;
}

extern "C" int expm_pfd_queue_stats_get(expm_pfd_queue_t q, expm_pfd_queue_stats* out) {
  if (!q || !out) return EXPM_PFD_ERR_NULL;
  std::lock_guard<std::mutex> lk(q->mu);
  expm_pfd_queue_stats s{};
  s.submitted = q->submitted;
  s.tridiag_requests = q->tri_requests;
  s.reductions = q->reductions;
  s.completed = q->completed;
  s.failed = q->failed;
  s.fallbacks = q->fallbacks;
  s.groups = q->groups;
  s.mean_group_size = q->groups ? (double)q->grouped / q->groups : 0.0;
  s.padded_up = q->padded_up;
  s.peak_bytes = q->peak;
  s.registered = (int64_t)q->mats.size();
  s.registered_bytes = q->mat_bytes;
  std::vector<double> v = q->lat_ms;
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) { return v[std::min(v.size() - 1, (size_t)std::llround(p * (v.size() - 1)))]; };
    s.p50_ms = pct(0.5);
    s.p99_ms = pct(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    s.mean_ms = sum / v.size();
    s.max_ms = v.back();
    const double span = std::chrono::duration<double>(q->last_done - q->first_submit).count();
    s.solves_per_s = span > 0 ? q->completed / span : 0.0;
  }
  *out = s;
  return 0;
}

extern "C" int expm_pfd_queue_destroy(expm_pfd_queue_t q) {
  if (!q) return EXPM_PFD_ERR_NULL;
  {
    std::lock_guard<std::mutex> lk(q->mu);
    q->stop = true;
    q->cv.notify_all();
  }
  q->worker.join();  // returns once every request has completed or failed
  {
    std::lock_guard<std::mutex> lk(q->mu);
    q->stop_waiters = true;
    q->cv_flight.notify_all();
  }
  for (auto& w : q->waiters) w.join();
  (void)hipDeviceSynchronize();
  for (auto& kv : q->free_plans)
    for (expm_pfd_plan_t p : kv.second) free_plan(p);
  for (auto& kv : q->mats) {
    (void)hipFreeAsync(kv.second.A, q->aux);
    if (kv.second.tri) tri_release(kv.second.tri, q->aux);
  }
  (void)hipStreamSynchronize(q->aux);
  for (auto& kv : q->mats) q->give_event(kv.second.ready);
  for (hipStream_t s : q->streams) (void)hipStreamSynchronize(s);
  for (hipStream_t s : q->streams) (void)hipStreamDestroy(s);
  for (hipEvent_t e : q->stream_ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : q->event_pool) (void)hipEventDestroy(e);
  (void)hipStreamDestroy(q->aux);
  (void)hipFree(q->dev_status);
  (void)hipHostFree(q->host_status);
  // the plans' workspace went back to the stream-ordered pool: hand it back to
  // the device
  hipMemPool_t mpool = nullptr;
  if (hipDeviceGetDefaultMemPool(&mpool, q->device) == hipSuccess) (void)hipMemPoolTrimTo(mpool, 0);
  (void)hipGetLastError();
  delete q;
  return 0;
}

extern "C" int expm_pfd_trace(int class_mask) {
  trace::clear();
  trace::mask = (unsigned)class_mask & ((1u << EXPM_PFD_K_COUNT) - 1u);
  return 0;
}

extern "C" int expm_pfd_trace_summary(int cls, double* ms, int64_t* launches, double* flops, double* bytes) {
  if (cls < 0 || cls >= EXPM_PFD_K_COUNT) return EXPM_PFD_ERR_ARG;
  double t = 0, f = 0, b = 0;
  int64_t k = 0;
  for (auto& r : trace::recs) {
    if (r.cls != cls) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return EXPM_PFD_ERR_HIP;
    float x = 0;
    if (hipEventElapsedTime(&x, r.a, r.b) != hipSuccess) return EXPM_PFD_ERR_HIP;
    t += x;
    f += r.flops;
    b += r.bytes;
    ++k;
  }
  if (ms) *ms = t;
  if (launches) *launches = k;
  if (flops) *flops = f;
  if (bytes) *bytes = b;
  return 0;
}

extern "C" const char* expm_pfd_strerror(int code) {
  switch (code) {
    case EXPM_PFD_OK: return "success";
    case EXPM_PFD_ERR_DEGREE: return "degree must be even and in [2, 64]";
    case EXPM_PFD_ERR_DIM: return "invalid dimension (n, m)";
    case EXPM_PFD_ERR_NULL: return "required pointer is NULL";
    case EXPM_PFD_ERR_LD: return "leading dimension smaller than the row count";
    case EXPM_PFD_ERR_OOM: return "device memory allocation failed";
    case EXPM_PFD_ERR_HIP: return "HIP runtime error";
    case EXPM_PFD_ERR_ARG: return "invalid argument";
    case EXPM_PFD_ERR_CONST: return "root finding for the constants did not converge";
    case EXPM_PFD_ERR_BUDGET: return "request exceeds the queue's HBM budget";
    case EXPM_PFD_ERR_TICKET: return "unknown ticket or matrix id";
    case EXPM_PFD_ERR_SYNC: return "a triangular sweep lost its dependency order; results are invalid";
    case EXPM_PFD_ERR_SCRATCH: return "the problem's workspace exceeds the fixed scratch array (EXPM_PFD_NOALLOC_BYTES)";
    default: return "unknown error";
  }
}

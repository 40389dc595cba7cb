// C ABI of the library (declared in include/lbm.h): host-side argument validation and
// dispatch to the kernels.  Every check runs before the first HIP call, so invalid
// arguments never reach the device.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "kernels.h"
#include "lattice.h"
#include "lbm.h"

namespace {

thread_local char g_last_error[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(LBM_EHIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

struct Geometry {
  int D = 0, Q = 0;
  size_t word = 0;  // bytes per stored population
  size_t real = 0;  // bytes per real (force, rho, u, adjoint)
  size_t pop = 0;   // entries of a population buffer: Q * pitch * ny * nz
  lbm::GridArgs args{};
};

uint32_t pick_block_x(int64_t nx) {
  // The row segment per block that leaves the fewest idle threads (ties: the longer).
  uint32_t best = 256;
  int64_t best_waste = -1;
  for (uint32_t bx : {256u, 128u, 64u}) {
    const int64_t waste = ((nx + bx - 1) / bx) * bx - nx;
    if (best_waste < 0 || waste < best_waste) {
      best = bx;
      best_waste = waste;
    }
  }
  return best;
}

int check_grid(const lbm_grid* g, Geometry* geo) {
  if (!g) return fail(LBM_ENULL, "grid is NULL");
  if (g->lattice != LBM_D2Q9 && g->lattice != LBM_D3Q19 && g->lattice != LBM_D3Q27)
    return fail(LBM_EINVAL, "unknown lattice %d", g->lattice);
  if (g->storage < LBM_F64 || g->storage > LBM_BF16S) return fail(LBM_EINVAL, "unknown storage %d", g->storage);
  if (g->nx < 1 || g->ny < 1 || g->nz < 1)
    return fail(LBM_EINVAL, "grid dimensions must be >= 1 (got %lld x %lld x %lld)", (long long)g->nx,
                (long long)g->ny, (long long)g->nz);
  if (g->lattice == LBM_D2Q9 && g->nz != 1) return fail(LBM_EINVAL, "D2Q9 needs nz == 1 (got %lld)", (long long)g->nz);
  const int64_t lim = 2147483647;
  if (g->nx > lim || g->ny > lim || g->nz > lim) return fail(LBM_ERANGE, "a grid dimension exceeds 2^31-1");
  if (g->nx * g->ny > lim || (g->nx * g->ny) * g->nz > lim)
    return fail(LBM_ERANGE, "grid has more than 2^31-1 cells");
  if (g->pitch != 0 && g->pitch < g->nx)
    return fail(LBM_EINVAL, "pitch must be 0 or >= nx (got %lld < %lld)", (long long)g->pitch, (long long)g->nx);
  if (g->pitch > lim) return fail(LBM_ERANGE, "pitch exceeds 2^31-1");
  geo->D = g->lattice == LBM_D2Q9 ? 2 : 3;
  geo->Q = g->lattice == LBM_D2Q9 ? 9 : g->lattice == LBM_D3Q19 ? 19 : 27;
  geo->word = g->storage == LBM_F64 ? 8 : (g->storage == LBM_F32 || g->storage == LBM_F32S) ? 4 : 2;
  geo->real = g->storage == LBM_F64 ? 8 : 4;
  geo->args.nx = (uint32_t)g->nx;
  geo->args.ny = (uint32_t)g->ny;
  geo->args.nz = (uint32_t)g->nz;
  geo->args.ncells = (uint64_t)(g->nx * g->ny * g->nz);
  geo->args.block_x = pick_block_x(g->nx);
  geo->args.z0 = 0;
  geo->args.nzl = (uint32_t)g->nz;
  geo->args.ghost = 0;
  geo->args.pitch = (uint32_t)(g->pitch ? g->pitch : g->nx);
  geo->pop = (size_t)geo->Q * geo->args.pitch * (size_t)g->ny * (size_t)g->nz;
  // Inside a row the kernels address a lane's word as a 32-bit byte offset from the
  // row base (populations, adjoint arrays and real fields alike), so a row of pitch
  // words of the widest element the grid uses must stay below 4 GiB.
  if ((uint64_t)geo->args.pitch * geo->real >= (uint64_t(1) << 32))
    return fail(LBM_ERANGE, "a row of %u words of %zu bytes spans 4 GiB or more (row offsets are 32-bit)",
                geo->args.pitch, geo->real);
  return LBM_OK;
}

int check_ptr(const void* p, const char* name, bool required) {
  if (!p) return required ? fail(LBM_ENULL, "%s is NULL", name) : LBM_OK;
  if (reinterpret_cast<uintptr_t>(p) % 16 != 0) return fail(LBM_EALIGN, "%s is not 16-byte aligned", name);
  return LBM_OK;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b || na == 0 || nb == 0) return false;
  const uintptr_t pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  return pa < pb + nb && pb < pa + na;
}

int check_tau(double tau) {
  if (!std::isfinite(tau) || !(tau > 0.5)) return fail(LBM_EINVAL, "tau must be finite and > 1/2 (got %g)", tau);
  return LBM_OK;
}


template <typename LT>
void fill_lattice(int* c, double* w) {
  for (int i = 0; i < LT::Q; ++i) {
    if (c) {
      c[i * LT::D + 0] = LT::cx(i);
      c[i * LT::D + 1] = LT::cy(i);
      if (LT::D == 3) c[i * LT::D + 2] = LT::cz(i);
    }
    if (w) w[i] = LT::w(i);
  }
}

// The directions crossing a z face: those with c_z == cz, which are consecutive in the
// lattice order (c_z varies slowest); returns the first index and the count.
template <typename LT>
void face_dirs_of(int cz, int* i0, int* n) {
  *i0 = -1;
  *n = 0;
  for (int i = 0; i < LT::Q; ++i)
    if (LT::cz(i) == cz) {
      if (*i0 < 0) *i0 = i;
      ++*n;
    }
}

void face_dirs(int lattice, int cz, int* i0, int* n) {
  if (lattice == LBM_D3Q19)
    face_dirs_of<lbm::Lattice<lbm::kD3Q19>>(cz, i0, n);
  else
    face_dirs_of<lbm::Lattice<lbm::kD3Q27>>(cz, i0, n);
}

#define LBM_TRY(expr)          \
  do {                         \
    const int rc_ = (expr);    \
    if (rc_ != LBM_OK) return rc_; \
  } while (0)

}  // namespace

extern "C" {

const char* lbm_strerror(int status) {
  switch (status) {
    case LBM_OK: return "success";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENULL: return "required pointer is NULL";
    case LBM_EALIGN: return "pointer is not 16-byte aligned";
    case LBM_EALIAS: return "output buffer overlaps an input buffer";
    case LBM_EUNSUP: return "unsupported combination of arguments";
    case LBM_ERANGE: return "grid too large";
    case LBM_EHIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* lbm_last_error(void) { return g_last_error; }

int lbm_version(void) { return 10100; }

int lbm_lattice_info(int lattice, int* D, int* Q, int* c, double* w) {
  switch (lattice) {
    case LBM_D2Q9:
      if (D) *D = 2;
      if (Q) *Q = 9;
      fill_lattice<lbm::Lattice<lbm::kD2Q9>>(c, w);
      return LBM_OK;
    case LBM_D3Q19:
      if (D) *D = 3;
      if (Q) *Q = 19;
      fill_lattice<lbm::Lattice<lbm::kD3Q19>>(c, w);
      return LBM_OK;
    case LBM_D3Q27:
      if (D) *D = 3;
      if (Q) *Q = 27;
      fill_lattice<lbm::Lattice<lbm::kD3Q27>>(c, w);
      return LBM_OK;
  }
  return fail(LBM_EINVAL, "unknown lattice %d", lattice);
}

int lbm_init_equilibrium(const lbm_grid* grid, const double* rho, const double* u, void* f_out, void* stream) {
  Geometry geo;
  LBM_TRY(check_grid(grid, &geo));
  LBM_TRY(check_ptr(rho, "rho", false));
  LBM_TRY(check_ptr(u, "u", true));
  LBM_TRY(check_ptr(f_out, "f_out", true));
  const size_t N = geo.args.ncells;
  const size_t fbytes = geo.pop * geo.word;
  if (overlap(f_out, fbytes, rho, N * 8) || overlap(f_out, fbytes, u, geo.D * N * 8))
    return fail(LBM_EALIAS, "f_out overlaps rho or u");
  const hipError_t e = lbm::launch_init(grid->lattice, grid->storage, rho, u, f_out, geo.args, (hipStream_t)stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_init_equilibrium launch");
}

}  // extern "C"

namespace {

// Launches of a call of n_steps: steps run four (D2Q9) or two at a time where a kernel
// takes the grid.  Each launch swaps the buffers, so the multi-step launches come in
// pairs of equal kind, which leaves the result where n_steps single steps leave it:
// n = 8 quads/2 + 4 pairs/2 + singles, with the singles (at most three) first.
struct Plan {
  int single, paired, quad;
};
Plan launch_plan(const lbm_grid* grid, const Geometry& geo, int n_steps) {
  const int most = lbm::max_steps_per_launch(grid->lattice, grid->storage, geo.args);
  Plan p{};
  p.quad = most >= 4 ? 2 * (n_steps / 8) : 0;
  const int rest = n_steps - 4 * p.quad;
  p.paired = most >= 2 ? 2 * (rest / 4) : 0;
  p.single = rest - 2 * p.paired;
  return p;
}

int step_common(const lbm_grid* grid, void* f_in, void* f_out, double tau, const void* field, int force_mode,
                int n_steps, void* stream, const char* name) {
  Geometry geo;
  LBM_TRY(check_grid(grid, &geo));
  LBM_TRY(check_tau(tau));
  if (n_steps < 1) return fail(LBM_EINVAL, "n_steps must be >= 1 (got %d)", n_steps);
  LBM_TRY(check_ptr(f_in, "f_in", true));
  LBM_TRY(check_ptr(f_out, "f_out", true));
  LBM_TRY(check_ptr(field, force_mode == lbm::kShiftForce ? "du" : "force", force_mode == lbm::kShiftForce));
  const size_t N = geo.args.ncells;
  const size_t fbytes = geo.pop * geo.word, vbytes = geo.D * N * geo.real;
  if (overlap(f_in, fbytes, f_out, fbytes)) return fail(LBM_EALIAS, "f_in and f_out overlap");
  if (overlap(field, vbytes, f_in, fbytes) || overlap(field, vbytes, f_out, fbytes))
    return fail(LBM_EALIAS, "the per-cell field overlaps a population buffer");
  const double omega = 1.0 / tau;
  const int mode = field ? force_mode : lbm::kNoForce;
  const Plan plan = launch_plan(grid, geo, n_steps);
  void* bufs[2] = {f_in, f_out};
  int cur = 0;
  for (int k = 0; k < plan.single; ++k, cur ^= 1) {
    const hipError_t e = lbm::launch_step(grid->lattice, grid->storage, bufs[cur], bufs[cur ^ 1], field, mode,
                                          geo.args, omega, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, name);
  }
  for (int nst : {2, 4}) {
    for (int k = 0; k < (nst == 2 ? plan.paired : plan.quad); ++k, cur ^= 1) {
      const hipError_t e = lbm::launch_stepn(grid->lattice, grid->storage, nst, bufs[cur], bufs[cur ^ 1], field,
                                             mode, geo.args, omega, (hipStream_t)stream);
      if (e != hipSuccess) return hip_fail(e, name);
    }
  }
  return (n_steps & 1) ? 0 : 1;
}

}  // namespace

extern "C" {

int lbm_step(const lbm_grid* grid, void* f_in, void* f_out, double tau, const void* force, int n_steps,
             void* stream) {
  return step_common(grid, f_in, f_out, tau, force, lbm::kGuoForce, n_steps, stream, "lbm_step launch");
}

int lbm_step_shifted(const lbm_grid* grid, void* f_in, void* f_out, double tau, const void* du, int n_steps,
                     void* stream) {
  return step_common(grid, f_in, f_out, tau, du, lbm::kShiftForce, n_steps, stream, "lbm_step_shifted launch");
}

int lbm_step_launches(const lbm_grid* grid, int n_steps, int* single, int* paired, int* quad) {
  Geometry geo;
  LBM_TRY(check_grid(grid, &geo));
  if (n_steps < 1) return fail(LBM_EINVAL, "n_steps must be >= 1 (got %d)", n_steps);
  if (!single || !paired || !quad) return fail(LBM_ENULL, "single, paired and quad must not be NULL");
  const Plan p = launch_plan(grid, geo, n_steps);
  *single = p.single;
  *paired = p.paired;
  *quad = p.quad;
  return LBM_OK;
}

}  // extern "C"

namespace {

// Shared validation and launch loop of the MRT entry points.
int mrt_common(const lbm_grid* grid, void* f_in, void* f_out, const double* taus, const void* ghost,
               size_t ghost_bytes, int ghost_mode, int n_steps, void* stream, const char* name) {
  Geometry geo;
  LBM_TRY(check_grid(grid, &geo));
  if (grid->lattice != LBM_D2Q9) return fail(LBM_EUNSUP, "%s supports D2Q9 only", name);
  if (n_steps < 1) return fail(LBM_EINVAL, "n_steps must be >= 1 (got %d)", n_steps);
  LBM_TRY(check_ptr(f_in, "f_in", true));
  LBM_TRY(check_ptr(f_out, "f_out", true));
  const size_t fbytes = geo.pop * geo.word;
  if (overlap(f_in, fbytes, f_out, fbytes)) return fail(LBM_EALIAS, "f_in and f_out overlap");
  if (overlap(ghost, ghost_bytes, f_in, fbytes) || overlap(ghost, ghost_bytes, f_out, fbytes))
    return fail(LBM_EALIAS, "the ghost-time source overlaps a population buffer");
  // |R_k|^2 of the w-orthogonal moment rows 3..8 (see mrt_step_kernel)
  const double norm2[6] = {2.0, 1.0 / 9.0, 2.0, 4.0, 8.0 / 3.0, 8.0 / 3.0};
  double scales[6];
  for (int k = 0; k < 6; ++k) scales[k] = 1.0 / (taus[k + 3] * norm2[k]);
  // uniform relaxation times or a ghost-time field: several steps per launch where
  // lbm_step would take them (lbm_step_launches); the network's times step singly
  const bool multi = ghost_mode == lbm::kGhostUniform || ghost_mode == lbm::kGhostField;
  const Plan plan = multi ? launch_plan(grid, geo, n_steps) : Plan{n_steps, 0, 0};
  void* bufs[2] = {f_in, f_out};
  int cur = 0;
  for (int k = 0; k < plan.single; ++k, cur ^= 1) {
    const hipError_t e = lbm::launch_mrt(grid->storage, bufs[cur], bufs[cur ^ 1], ghost, ghost_mode, geo.args, scales,
                                         (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, name);
  }
  for (int nst : {2, 4}) {
    for (int k = 0; k < (nst == 2 ? plan.paired : plan.quad); ++k, cur ^= 1) {
      const hipError_t e = lbm::launch_stepn_mrt(grid->storage, nst, bufs[cur], bufs[cur ^ 1], geo.args, scales,
                                                 ghost_mode == lbm::kGhostField ? ghost : nullptr, (hipStream_t)stream);
      if (e != hipSuccess) return hip_fail(e, name);
    }
  }
  return (n_steps & 1) ? 0 : 1;
}

}  // namespace

extern "C" {

int lbm_step_mrt(const lbm_grid* grid, void* f_in, void* f_out, const double* tau_moments, const void* tau_ghost,
                 int n_steps, void* stream) {
  Geometry geo;
  LBM_TRY(check_grid(grid, &geo));
  if (!tau_moments) return fail(LBM_ENULL, "tau_moments is NULL");
  for (int k = 3; k < 9; ++k) LBM_TRY(check_tau(tau_moments[k]));
  LBM_TRY(check_ptr(tau_ghost, "tau_ghost", false));
  return mrt_common(grid, f_in, f_out, tau_moments, tau_ghost, 3 * geo.args.ncells * geo.real,
                    tau_ghost ? lbm::kGhostField : lbm::kGhostUniform, n_steps, stream, "lbm_step_mrt");
}

int lbm_step_neural(const lbm_grid* grid, void* f_in, void* f_out, double tau_shear, const void* params,
                    int activation, int n_steps, void* stream) {
  Geometry geo;
  LBM_TRY(check_grid(grid, &geo));
  LBM_TRY(check_tau(tau_shear));
  if (activation != LBM_ACT_RELU && activation != LBM_ACT_TANH)
    return fail(LBM_EINVAL, "activation must be LBM_ACT_RELU or LBM_ACT_TANH (got %d)", activation);
  LBM_TRY(check_ptr(params, "params", true));
  // tau_6..8 come from the network; these uniform values are not used
  const double taus[9] = {1, 1, 1, tau_shear, tau_shear, tau_shear, 1, 1, 1};
  return mrt_common(grid, f_in, f_out, taus, params, (size_t)lbm::kNeuralParams * geo.real,
                    activation == LBM_ACT_RELU ? lbm::kGhostRelu : lbm::kGhostTanh, n_steps, stream,
                    "lbm_step_neural");
}

int lbm_step_slab(const lbm_grid* slab, const void* f_in, void* f_out, double tau, const void* force,
                  int64_t z_begin, int64_t z_end, void* stream) {
  Geometry geo;
  LBM_TRY(check_grid(slab, &geo));
  if (geo.D != 3) return fail(LBM_EUNSUP, "lbm_step_slab needs a 3D lattice (z-slabs)");
  LBM_TRY(check_tau(tau));
  if (z_begin < 0 || z_end > slab->nz || z_begin >= z_end)
    return fail(LBM_EINVAL, "plane range [%lld, %lld) is empty or outside [0, %lld)", (long long)z_begin,
                (long long)z_end, (long long)slab->nz);
  LBM_TRY(check_ptr(f_in, "f_in", true));
  LBM_TRY(check_ptr(f_out, "f_out", true));
  LBM_TRY(check_ptr(force, "force", false));
  const size_t plane = (size_t)geo.Q * geo.args.pitch * geo.args.ny * geo.word;
  const size_t fbytes = plane * (size_t)(slab->nz + 2), vbytes = geo.D * geo.args.ncells * geo.real;
  if (overlap(f_in, fbytes, f_out, fbytes)) return fail(LBM_EALIAS, "f_in and f_out overlap");
  if (overlap(force, vbytes, f_in, fbytes) || overlap(force, vbytes, f_out, fbytes))
    return fail(LBM_EALIAS, "force overlaps a population buffer");
  geo.args.z0 = (uint32_t)z_begin;
  geo.args.nzl = (uint32_t)(z_end - z_begin);
  geo.args.ghost = 1;
  const hipError_t e = lbm::launch_step(slab->lattice, slab->storage, f_in, f_out, force,
                                        force ? lbm::kGuoForce : lbm::kNoForce, geo.args, 1.0 / tau,
                                        (hipStream_t)stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_step_slab launch");
}

int lbm_slab_halo_copy(const lbm_grid* src_slab, const void* src, const lbm_grid* dst_slab, void* dst, int face,
                       void* stream) {
  Geometry gs, gd;
  LBM_TRY(check_grid(src_slab, &gs));
  LBM_TRY(check_grid(dst_slab, &gd));
  if (gs.D != 3) return fail(LBM_EUNSUP, "lbm_slab_halo_copy needs a 3D lattice (z-slabs)");
  if (src_slab->lattice != dst_slab->lattice || src_slab->storage != dst_slab->storage ||
      src_slab->nx != dst_slab->nx || src_slab->ny != dst_slab->ny || gs.args.pitch != gd.args.pitch)
    return fail(LBM_EINVAL, "source and destination slabs differ in lattice, storage, nx, ny or pitch");
  if (face != LBM_FACE_LOW && face != LBM_FACE_HIGH) return fail(LBM_EINVAL, "face must be 0 or 1 (got %d)", face);
  LBM_TRY(check_ptr(src, "src", true));
  LBM_TRY(check_ptr(dst, "dst", true));
  // LOW: src's lowest interior plane (buffer plane 1), directions with c_z = -1, into dst's
  // upper ghost plane (nz + 1).  HIGH: src's highest interior plane (nz), c_z = +1, into
  // dst's lower ghost plane (0).
  const uint64_t src_plane = face == LBM_FACE_LOW ? 1 : (uint64_t)src_slab->nz;
  const uint64_t dst_plane = face == LBM_FACE_LOW ? (uint64_t)dst_slab->nz + 1 : 0;
  int i0 = 0, n = 0;
  face_dirs(src_slab->lattice, face == LBM_FACE_LOW ? -1 : 1, &i0, &n);
  const size_t plane = (size_t)gs.Q * gs.args.pitch * gs.args.ny * gs.word;
  if (overlap((const char*)src + src_plane * plane, plane, (const char*)dst + dst_plane * plane, plane))
    return fail(LBM_EALIAS, "the source plane overlaps the destination ghost plane");
  const hipError_t e = lbm::launch_halo_copy(gs.Q, (int)gs.word, src, src_plane, dst, dst_plane, i0, n, gs.args.pitch,
                                             gs.args.ny, (hipStream_t)stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_slab_halo_copy launch");
}

int lbm_step_slab2_available(const lbm_grid* slab, int* available) {
  Geometry geo;
  LBM_TRY(check_grid(slab, &geo));
  if (!available) return fail(LBM_ENULL, "available is NULL");
  geo.args.ghost = 2;
  *available = geo.D == 3 && lbm::step2_slab_supported(slab->lattice, slab->storage, geo.args) ? 1 : 0;
  return LBM_OK;
}

int lbm_step_slab2(const lbm_grid* slab, const void* f_in, void* f_out, double tau, const void* force,
                   int64_t z_begin, int64_t z_end, void* stream) {
  Geometry geo;
  LBM_TRY(check_grid(slab, &geo));
  if (geo.D != 3) return fail(LBM_EUNSUP, "lbm_step_slab2 needs a 3D lattice (z-slabs)");
  LBM_TRY(check_tau(tau));
  if (slab->nz < 2) return fail(LBM_EINVAL, "a slab of two-step launches needs nz >= 2 (got %lld)", (long long)slab->nz);
  if (z_begin < 0 || z_end > slab->nz || z_begin >= z_end)
    return fail(LBM_EINVAL, "plane range [%lld, %lld) is empty or outside [0, %lld)", (long long)z_begin,
                (long long)z_end, (long long)slab->nz);
  LBM_TRY(check_ptr(f_in, "f_in", true));
  LBM_TRY(check_ptr(f_out, "f_out", true));
  LBM_TRY(check_ptr(force, "force", false));
  const size_t plane = (size_t)geo.Q * geo.args.pitch * geo.args.ny * geo.word;
  const size_t fbytes = plane * (size_t)(slab->nz + 4);
  const size_t vbytes = (size_t)geo.D * geo.args.nx * geo.args.ny * (size_t)(slab->nz + 2) * geo.real;
  if (overlap(f_in, fbytes, f_out, fbytes)) return fail(LBM_EALIAS, "f_in and f_out overlap");
  if (overlap(force, vbytes, f_in, fbytes) || overlap(force, vbytes, f_out, fbytes))
    return fail(LBM_EALIAS, "force overlaps a population buffer");
  geo.args.ghost = 2;
  geo.args.z0 = (uint32_t)z_begin;
  geo.args.nzl = (uint32_t)(z_end - z_begin);
  if (!lbm::step2_slab_supported(slab->lattice, slab->storage, geo.args))
    return fail(LBM_EUNSUP, "two steps per launch do not take this slab or storage kind "
                            "(lbm_step_slab2_available)");
  const hipError_t e = lbm::launch_step2_slab(slab->lattice, slab->storage, f_in, f_out, force,
                                              force ? lbm::kGuoForce : lbm::kNoForce, geo.args, 1.0 / tau,
                                              (hipStream_t)stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_step_slab2 launch");
}

int lbm_slab2_halo_copy(const lbm_grid* src_slab, const void* src, const lbm_grid* dst_slab, void* dst, int face,
                        void* stream) {
  Geometry gs, gd;
  LBM_TRY(check_grid(src_slab, &gs));
  LBM_TRY(check_grid(dst_slab, &gd));
  if (gs.D != 3) return fail(LBM_EUNSUP, "lbm_slab2_halo_copy needs a 3D lattice (z-slabs)");
  if (src_slab->lattice != dst_slab->lattice || src_slab->storage != dst_slab->storage ||
      src_slab->nx != dst_slab->nx || src_slab->ny != dst_slab->ny || gs.args.pitch != gd.args.pitch)
    return fail(LBM_EINVAL, "source and destination slabs differ in lattice, storage, nx, ny or pitch");
  if (face != LBM_FACE_LOW && face != LBM_FACE_HIGH) return fail(LBM_EINVAL, "face must be 0 or 1 (got %d)", face);
  if (src_slab->nz < 2 || dst_slab->nz < 2) return fail(LBM_EINVAL, "slabs of two-step launches need nz >= 2");
  LBM_TRY(check_ptr(src, "src", true));
  LBM_TRY(check_ptr(dst, "dst", true));
  // Buffer plane p + 2 holds slab plane p.  LOW: src planes 0 (c_z = -1 and 0) and 1
  // (c_z = -1) into dst's ghost planes nz and nz + 1.  HIGH: src planes nz - 1 (c_z = 0
  // and +1) and nz - 2 (c_z = +1) into dst's ghost planes -1 and -2.
  const bool low = face == LBM_FACE_LOW;
  const int64_t ns = src_slab->nz, nd = dst_slab->nz;
  int im, nm, i0, n0, ip, np;
  face_dirs(src_slab->lattice, -1, &im, &nm);
  face_dirs(src_slab->lattice, 0, &i0, &n0);
  face_dirs(src_slab->lattice, 1, &ip, &np);
  if (i0 != im + nm || ip != i0 + n0) return fail(LBM_EINVAL, "direction groups are not consecutive");
  struct Part {
    uint64_t src_plane, dst_plane;
    int first, count;
  };
  const Part parts[2] = {
      low ? Part{2, (uint64_t)nd + 2, im, nm + n0} : Part{(uint64_t)ns + 1, 1, i0, n0 + np},
      low ? Part{3, (uint64_t)nd + 3, im, nm} : Part{(uint64_t)ns, 0, ip, np},
  };
  const size_t plane = (size_t)gs.Q * gs.args.pitch * gs.args.ny * gs.word;
  for (const Part& q : parts)
    for (const Part& r : parts)
      if (overlap((const char*)src + q.src_plane * plane, plane, (const char*)dst + r.dst_plane * plane, plane))
        return fail(LBM_EALIAS, "a source plane overlaps a destination ghost plane");
  for (const Part& q : parts) {
    const hipError_t e = lbm::launch_halo_copy(gs.Q, (int)gs.word, src, q.src_plane, dst, q.dst_plane, q.first,
                                               q.count, gs.args.pitch, gs.args.ny, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "lbm_slab2_halo_copy launch");
  }
  return LBM_OK;
}

int lbm_stream_only(const lbm_grid* grid, const void* f_in, void* f_out, void* stream) {
  Geometry geo;
  LBM_TRY(check_grid(grid, &geo));
  LBM_TRY(check_ptr(f_in, "f_in", true));
  LBM_TRY(check_ptr(f_out, "f_out", true));
  const size_t fbytes = geo.pop * geo.word;
  if (overlap(f_in, fbytes, f_out, fbytes)) return fail(LBM_EALIAS, "f_in and f_out overlap");
  const hipError_t e = lbm::launch_stream(grid->lattice, (int)geo.word, f_in, f_out, geo.args, (hipStream_t)stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_stream_only launch");
}

int lbm_copy(const void* src, void* dst, size_t bytes, void* stream) {
  LBM_TRY(check_ptr(src, "src", true));
  LBM_TRY(check_ptr(dst, "dst", true));
  if (bytes % 16 != 0) return fail(LBM_EINVAL, "bytes must be a multiple of 16 (got %zu)", bytes);
  if (bytes / 16 > (size_t)0xFFFFFFFF * 256) return fail(LBM_ERANGE, "copy too large");
  if (overlap(src, bytes, dst, bytes)) return fail(LBM_EALIAS, "src and dst overlap");
  const hipError_t e = lbm::launch_copy16(src, dst, bytes / 16, (hipStream_t)stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_copy launch");
}

int lbm_moments_workspace_size(const lbm_grid* grid, size_t* bytes) {
  Geometry geo;
  LBM_TRY(check_grid(grid, &geo));
  if (!bytes) return fail(LBM_ENULL, "bytes is NULL");
  *bytes = (size_t)lbm::moments_workspace_entries(geo.args) * lbm::kNred * sizeof(double);
  return LBM_OK;
}

int lbm_moments(const lbm_grid* grid, const void* g, const void* force, void* rho_out, void* u_out, double* red,
                void* workspace, size_t workspace_bytes, void* stream) {
  Geometry geo;
  LBM_TRY(check_grid(grid, &geo));
  LBM_TRY(check_ptr(g, "g", true));
  LBM_TRY(check_ptr(force, "force", false));
  LBM_TRY(check_ptr(rho_out, "rho_out", false));
  LBM_TRY(check_ptr(u_out, "u_out", false));
  LBM_TRY(check_ptr(red, "red", false));
  const size_t need = (size_t)lbm::moments_workspace_entries(geo.args) * lbm::kNred * sizeof(double);
  if (red) {
    LBM_TRY(check_ptr(workspace, "workspace", true));
    if (workspace_bytes < need)
      return fail(LBM_EINVAL, "workspace has %zu bytes, lbm_moments needs %zu", workspace_bytes, need);
  }
  const size_t N = geo.args.ncells;
  const size_t fbytes = geo.pop * geo.word;
  const size_t rbytes = N * geo.real, ubytes = geo.D * N * geo.real;
  const void* ins[2] = {g, force};
  const size_t insz[2] = {fbytes, geo.D * N * geo.real};
  void* outs[4] = {rho_out, u_out, red, red ? workspace : nullptr};
  const size_t outsz[4] = {rbytes, ubytes, lbm::kNred * sizeof(double), need};
  for (int a = 0; a < 4; ++a) {
    for (int b = 0; b < 2; ++b)
      if (overlap(outs[a], outsz[a], ins[b], insz[b])) return fail(LBM_EALIAS, "an output of lbm_moments overlaps an input");
    for (int b = a + 1; b < 4; ++b)
      if (overlap(outs[a], outsz[a], outs[b], outsz[b])) return fail(LBM_EALIAS, "two outputs of lbm_moments overlap");
  }
  const hipError_t e = lbm::launch_moments(grid->lattice, grid->storage, g, force, rho_out, u_out,
                                           red ? (double*)workspace : nullptr, red, geo.args, (hipStream_t)stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_moments launch");
}

}  // extern "C"

// ---------------------------------------------------------------------------------
// Fixed device scratch of lbm_moments_noalloc: the reduction partials live in this
// file-scope array (one copy per GPU, kept until the process ends) instead of a caller
// workspace.  In host code `scratch` only names the symbol; its device address on the
// current GPU comes from hipGetSymbolAddress, looked up once per device on the first
// call there and kept in g_scratch_dev.
// ---------------------------------------------------------------------------------
static constexpr uint64_t kScratchEntries = 131072;  // kNred doubles each: 8 MiB
static __device__ __align__(256) double scratch[kScratchEntries * lbm::kNred];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

int scratch_on_current_device(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(LBM_EUNSUP, "device ordinal %d beyond %d", dev, kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_dev[dev] = p;
  }
  *out = static_cast<double*>(g_scratch_dev[dev]);
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_moments_noalloc(const lbm_grid* grid, const void* g, const void* force, void* rho_out, void* u_out,
                        double* red, void* stream) {
  Geometry geo;
  LBM_TRY(check_grid(grid, &geo));
  LBM_TRY(check_ptr(g, "g", true));
  LBM_TRY(check_ptr(force, "force", false));
  LBM_TRY(check_ptr(rho_out, "rho_out", false));
  LBM_TRY(check_ptr(u_out, "u_out", false));
  LBM_TRY(check_ptr(red, "red", false));
  const bool fields = rho_out || u_out;
  const uint64_t need = red ? lbm::moments_entries_used(grid->lattice, geo.args, fields) : 0;
  if (need > kScratchEntries)
    return fail(LBM_ERANGE, "the reduction needs %llu partials, the fixed scratch holds %llu (use lbm_moments)",
                (unsigned long long)need, (unsigned long long)kScratchEntries);
  const size_t N = geo.args.ncells;
  const size_t fbytes = geo.pop * geo.word;
  const size_t rbytes = N * geo.real, ubytes = geo.D * N * geo.real;
  const void* ins[2] = {g, force};
  const size_t insz[2] = {fbytes, geo.D * N * geo.real};
  void* outs[3] = {rho_out, u_out, red};
  const size_t outsz[3] = {rbytes, ubytes, lbm::kNred * sizeof(double)};
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 2; ++b)
      if (overlap(outs[a], outsz[a], ins[b], insz[b]))
        return fail(LBM_EALIAS, "an output of lbm_moments_noalloc overlaps an input");
    for (int b = a + 1; b < 3; ++b)
      if (overlap(outs[a], outsz[a], outs[b], outsz[b]))
        return fail(LBM_EALIAS, "two outputs of lbm_moments_noalloc overlap");
  }
  double* ws = nullptr;
  if (red) LBM_TRY(scratch_on_current_device(&ws));
  const hipError_t e = lbm::launch_moments(grid->lattice, grid->storage, g, force, rho_out, u_out, ws, red, geo.args,
                                           (hipStream_t)stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_moments_noalloc launch");
}

}  // extern "C"

namespace {

// Shared validation of the three adjoint-step forms; `in_gathered` says whether adj_next
// is read at shifted addresses (all forms read g_t shifted).
int adjoint_common(const lbm_grid* grid, const void* g_t, const void* adj_next, void* adj_out, double tau,
                   const void* force, void* dforce, int mode, void* stream, const char* name) {
  Geometry geo;
  LBM_TRY(check_grid(grid, &geo));
  LBM_TRY(check_tau(tau));
  LBM_TRY(check_ptr(g_t, "g_t", true));
  LBM_TRY(check_ptr(adj_next, "adjoint input", true));
  LBM_TRY(check_ptr(adj_out, "adjoint output", true));
  LBM_TRY(check_ptr(force, "force", false));
  LBM_TRY(check_ptr(dforce, "dforce", false));
  if (dforce && !force) return fail(LBM_EUNSUP, "dforce needs the force the step used");
  const size_t N = geo.args.ncells;
  const size_t gbytes = geo.pop * geo.word, lbytes = geo.pop * geo.real, fbytes = geo.D * N * geo.real;
  if (overlap(adj_out, lbytes, g_t, gbytes) || overlap(adj_out, lbytes, adj_next, lbytes) ||
      overlap(adj_out, lbytes, force, fbytes) || overlap(adj_out, lbytes, dforce, fbytes))
    return fail(LBM_EALIAS, "the adjoint output overlaps another argument");
  if (overlap(dforce, fbytes, g_t, gbytes) || overlap(dforce, fbytes, adj_next, lbytes) ||
      overlap(dforce, fbytes, force, fbytes))
    return fail(LBM_EALIAS, "dforce overlaps another argument");
  const hipError_t e = lbm::launch_adjoint(grid->lattice, grid->storage, mode, g_t, adj_next, adj_out, force, dforce,
                                           geo.args, 1.0 / tau, (hipStream_t)stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, name);
}

}  // namespace

extern "C" {

int lbm_adjoint_step(const lbm_grid* grid, const void* g_t, const void* lam_next, void* lam_out, double tau,
                     const void* force, void* dforce, void* stream) {
  return adjoint_common(grid, g_t, lam_next, lam_out, tau, force, dforce, lbm::kAdjScatter, stream,
                        "lbm_adjoint_step launch");
}

int lbm_adjoint_step_local(const lbm_grid* grid, const void* g_t, const void* adj_next, int adj_is_chi,
                           void* chi_out, double tau, const void* force, void* dforce, void* stream) {
  if (adj_is_chi != 0 && adj_is_chi != 1) return fail(LBM_EINVAL, "adj_is_chi must be 0 or 1 (got %d)", adj_is_chi);
  return adjoint_common(grid, g_t, adj_next, chi_out, tau, force, dforce,
                        adj_is_chi ? lbm::kAdjLocalChi : lbm::kAdjLocalLam, stream, "lbm_adjoint_step_local launch");
}

int lbm_adjoint_step2_available(const lbm_grid* grid, int* available) {
  Geometry geo;
  LBM_TRY(check_grid(grid, &geo));
  if (!available) return fail(LBM_ENULL, "available is NULL");
  *available = lbm::adjoint2_supported(grid->lattice, grid->storage, geo.args) ? 1 : 0;
  return LBM_OK;
}

int lbm_adjoint_step2_local(const lbm_grid* grid, const void* g_t, const void* g_tm1, const void* chi_next,
                            void* chi_out, double tau, const void* force, void* dforce, void* stream) {
  Geometry geo;
  LBM_TRY(check_grid(grid, &geo));
  LBM_TRY(check_tau(tau));
  LBM_TRY(check_ptr(g_t, "g_t", true));
  LBM_TRY(check_ptr(g_tm1, "g_tm1", true));
  LBM_TRY(check_ptr(chi_next, "chi_next", true));
  LBM_TRY(check_ptr(chi_out, "chi_out", true));
  LBM_TRY(check_ptr(force, "force", false));
  LBM_TRY(check_ptr(dforce, "dforce", false));
  if (dforce && !force) return fail(LBM_EUNSUP, "dforce needs the force the steps used");
  if (!lbm::adjoint2_supported(grid->lattice, grid->storage, geo.args))
    return fail(LBM_EUNSUP, "two adjoint steps per launch do not take this grid or storage kind "
                            "(lbm_adjoint_step2_available)");
  const size_t N = geo.args.ncells;
  const size_t gbytes = geo.pop * geo.word, lbytes = geo.pop * geo.real, fbytes = geo.D * N * geo.real;
  if (overlap(chi_out, lbytes, g_t, gbytes) || overlap(chi_out, lbytes, g_tm1, gbytes) ||
      overlap(chi_out, lbytes, chi_next, lbytes) || overlap(chi_out, lbytes, force, fbytes) ||
      overlap(chi_out, lbytes, dforce, fbytes))
    return fail(LBM_EALIAS, "chi_out overlaps another argument");
  if (overlap(dforce, fbytes, g_t, gbytes) || overlap(dforce, fbytes, g_tm1, gbytes) ||
      overlap(dforce, fbytes, chi_next, lbytes) || overlap(dforce, fbytes, force, fbytes))
    return fail(LBM_EALIAS, "dforce overlaps another argument");
  const hipError_t e = lbm::launch_adjoint2(grid->lattice, grid->storage, g_t, g_tm1, chi_next, chi_out, force, dforce,
                                            geo.args, 1.0 / tau, (hipStream_t)stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_adjoint_step2_local launch");
}

int lbm_adjoint_unstream(const lbm_grid* grid, const void* chi, void* lam_out, void* stream) {
  Geometry geo;
  LBM_TRY(check_grid(grid, &geo));
  LBM_TRY(check_ptr(chi, "chi", true));
  LBM_TRY(check_ptr(lam_out, "lam_out", true));
  const size_t lbytes = geo.pop * geo.real;
  if (overlap(chi, lbytes, lam_out, lbytes)) return fail(LBM_EALIAS, "chi and lam_out overlap");
  const hipError_t e = lbm::launch_unstream(grid->lattice, (int)geo.real, chi, lam_out, geo.args, (hipStream_t)stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_adjoint_unstream launch");
}

int lbm_moments_adjoint(const lbm_grid* grid, const void* g, const void* force, const void* dL_drho,
                        const void* dL_du, void* lam_out, void* dforce, void* stream) {
  Geometry geo;
  LBM_TRY(check_grid(grid, &geo));
  LBM_TRY(check_ptr(g, "g", true));
  LBM_TRY(check_ptr(force, "force", false));
  LBM_TRY(check_ptr(dL_drho, "dL_drho", false));
  LBM_TRY(check_ptr(dL_du, "dL_du", false));
  LBM_TRY(check_ptr(lam_out, "lam_out", true));
  LBM_TRY(check_ptr(dforce, "dforce", false));
  if (dforce && !force) return fail(LBM_EUNSUP, "dforce needs the force the moments used");
  const size_t N = geo.args.ncells;
  const size_t gbytes = geo.pop * geo.word, lbytes = geo.pop * geo.real, vbytes = geo.D * N * geo.real;
  if (overlap(lam_out, lbytes, g, gbytes) || overlap(lam_out, lbytes, force, vbytes) ||
      overlap(lam_out, lbytes, dL_drho, N * geo.real) || overlap(lam_out, lbytes, dL_du, vbytes) ||
      overlap(lam_out, lbytes, dforce, vbytes))
    return fail(LBM_EALIAS, "lam_out overlaps another argument");
  if (overlap(dforce, vbytes, g, gbytes) || overlap(dforce, vbytes, force, vbytes) ||
      overlap(dforce, vbytes, dL_drho, N * geo.real) || overlap(dforce, vbytes, dL_du, vbytes))
    return fail(LBM_EALIAS, "dforce overlaps another argument");
  const hipError_t e = lbm::launch_moments_adjoint(grid->lattice, grid->storage, g, force, dL_drho, dL_du, lam_out,
                                                   dforce, geo.args, (hipStream_t)stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_moments_adjoint launch");
}

static int check_shells(const lbm_shells* sh, int D) {
  if (!sh) return fail(LBM_ENULL, "shells is NULL");
  if (D < 1 || D > 3) return fail(LBM_EINVAL, "D must be 1, 2 or 3 (got %d)", D);
  if (sh->n < 1 || sh->nshell < 1) return fail(LBM_EINVAL, "shells need n >= 1 and nshell >= 1");
  if (sh->n > 2147483647) return fail(LBM_ERANGE, "more than 2^31-1 wavevectors");
  LBM_TRY(check_ptr(sh->order, "shells.order", true));
  LBM_TRY(check_ptr(sh->offsets, "shells.offsets", true));
  LBM_TRY(check_ptr(sh->shell, "shells.shell", true));
  return LBM_OK;
}

// An output of the loss-head calls may not overlap the shell table it is computed with.
static bool overlaps_table(const lbm_shells* sh, const void* p, size_t bytes) {
  const size_t nb = (size_t)sh->n * 4, ob = ((size_t)sh->nshell + 1) * 4;
  return overlap(p, bytes, sh->order, nb) || overlap(p, bytes, sh->offsets, ob) || overlap(p, bytes, sh->shell, nb);
}

int lbm_shell_energy(const lbm_shells* shells, int D, const void* uhat, double scale, double* E, void* stream) {
  LBM_TRY(check_shells(shells, D));
  LBM_TRY(check_ptr(uhat, "uhat", true));
  LBM_TRY(check_ptr(E, "E", true));
  if (!std::isfinite(scale)) return fail(LBM_EINVAL, "scale must be finite");
  const size_t nb = (size_t)D * (size_t)shells->n * 16;
  if (overlap(uhat, nb, E, (size_t)shells->nshell * 8)) return fail(LBM_EALIAS, "E overlaps uhat");
  if (overlaps_table(shells, E, (size_t)shells->nshell * 8)) return fail(LBM_EALIAS, "E overlaps the shell table");
  const hipError_t e = lbm::launch_shell_energy(uhat, D, (uint32_t)shells->n, shells->order, shells->offsets,
                                                shells->nshell, scale, E, (hipStream_t)stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_shell_energy launch");
}

int lbm_log_spectrum_grad(const lbm_shells* shells, int D, void* uhat, const double* E, const double* E_target,
                          int k_lo, int k_hi, double cutoff, double scale, double* R, void* stream) {
  LBM_TRY(check_shells(shells, D));
  LBM_TRY(check_ptr(uhat, "uhat", true));
  LBM_TRY(check_ptr(E, "E", true));
  LBM_TRY(check_ptr(E_target, "E_target", true));
  LBM_TRY(check_ptr(R, "R", false));
  if (k_lo < 0 || k_hi < k_lo || k_hi >= shells->nshell)
    return fail(LBM_EINVAL, "need 0 <= k_lo <= k_hi < nshell (got %d, %d, %d)", k_lo, k_hi, shells->nshell);
  if (!std::isfinite(cutoff) || !(cutoff > 0)) return fail(LBM_EINVAL, "cutoff must be finite and > 0");
  if (!std::isfinite(scale)) return fail(LBM_EINVAL, "scale must be finite");
  const size_t nb = (size_t)D * (size_t)shells->n * 16, eb = (size_t)shells->nshell * 8;
  if (overlap(uhat, nb, E, eb) || overlap(uhat, nb, E_target, eb) || overlap(uhat, nb, R, 8))
    return fail(LBM_EALIAS, "uhat overlaps E, E_target or R");
  if (overlaps_table(shells, uhat, nb) || overlaps_table(shells, R, 8))
    return fail(LBM_EALIAS, "uhat or R overlaps the shell table");
  if (overlap(R, 8, E, eb) || overlap(R, 8, E_target, eb)) return fail(LBM_EALIAS, "R overlaps E or E_target");
  const hipError_t e =
      lbm::launch_log_spectrum_grad(uhat, D, (uint32_t)shells->n, shells->shell, E, E_target, shells->nshell, k_lo,
                                    k_hi, cutoff, scale, R, (hipStream_t)stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_log_spectrum_grad launch");
}

int lbm_real_part(const void* z, int64_t count, double scale, void* out, int out_storage, void* stream) {
  LBM_TRY(check_ptr(z, "z", true));
  LBM_TRY(check_ptr(out, "out", true));
  if (count < 1) return fail(LBM_EINVAL, "count must be >= 1");
  if (count > (int64_t)0xFFFFFFFF * 256) return fail(LBM_ERANGE, "count too large");
  if (out_storage != LBM_F32 && out_storage != LBM_F64)
    return fail(LBM_EINVAL, "out_storage must be LBM_F32 or LBM_F64 (got %d)", out_storage);
  if (!std::isfinite(scale)) return fail(LBM_EINVAL, "scale must be finite");
  const size_t ob = (size_t)count * (out_storage == LBM_F64 ? 8 : 4);
  if (overlap(z, (size_t)count * 16, out, ob)) return fail(LBM_EALIAS, "out overlaps z");
  const hipError_t e = lbm::launch_real_part(z, (uint64_t)count, scale, out, out_storage == LBM_F64,
                                             (hipStream_t)stream);
  return e == hipSuccess ? LBM_OK : hip_fail(e, "lbm_real_part launch");
}

}  // extern "C"

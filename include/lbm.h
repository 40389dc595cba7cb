/*
 * lbm.h - C ABI of the MI355X (gfx950) lattice-Boltzmann stream-and-collide library.
 *
 * The library implements one time step of the lattice Boltzmann method with the BGK
 * collision operator (Bedrunka et al., "Lettuce: PyTorch-based Lattice Boltzmann
 * Framework", arXiv:2106.12929, Sec. 2.1):
 *   Eq. 1  f_i(x + c_i, t + 1) = f_i(x, t) + Omega_i(f(x, t))        (stream + collide)
 *   Eq. 2  Omega_i = -(f_i - f_i^eq) / tau                            (BGK)
 *   Eq. 3  f_i^eq = w_i rho (1 + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u.u)   (c_s^2 = 1/3)
 *   Eq. 4  rho = sum_i f_i,   rho u = sum_i c_i f_i
 * on fully periodic D2Q9, D3Q19 and D3Q27 grids, with an optional per-cell body force (Guo
 * scheme, textbook), plus the reverse-mode derivative of the step (the automatic
 * differentiation of Sec. 3.2, written by hand).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice velocity order: c_i in {-1,0,1}^D with c_x fastest, then c_y, then c_z:
 *   i = 3(c_y+1) + (c_x+1)  (D2Q9),   i = 9(c_z+1) + 3(c_y+1) + (c_x+1)  (D3Q27);
 *   D3Q19 is the D3Q27 order without the 8 corner velocities (|c|^2 = 3).
 *   The rest velocity is i = Q/2 and the opposite of i is Q-1-i.  lbm_lattice_info()
 *   publishes c and w.
 *
 * Grid: nx, ny, nz >= 1 cells (nz = 1 for D2Q9), N = nx*ny*nz <= 2^31 - 1, and a row
 *   below 4 GiB: pitch * r < 2^32 bytes with r = 8 for LBM_F64 and r = 4 otherwise (the
 *   width of the grid's real type, its widest element), i.e. nx (or pitch) < 2^29
 *   for LBM_F64 and < 2^30 for the other kinds.  The kernels address a word inside a
 *   row by a 32-bit byte offset from the row's base.
 *   Cell (x, y, z) has linear index n = (z*ny + y)*nx + x (x fastest).
 *
 * Population buffers ("f", "g"): row-interleaved SoA.  The grid is nz*ny rows of nx
 *   cells; row r = z*ny + y holds its Q direction rows one after the other, so word
 *   (i, x, y, z) sits at ((z*ny + y)*Q + i)*nx + x, Q*N words in all (with a row pitch,
 *   see lbm_grid, nx is replaced by the pitch in both).  Each direction is contiguous
 *   along x within a row.  The word type and meaning depend on the
 *   storage kind:
 *     LBM_F64    double   f_i
 *     LBM_F32    float    f_i
 *     LBM_F32S   float    f_i - w_i         ("shifted": the deviation from rest)
 *     LBM_F16S   binary16 f_i - w_i  (raw 16-bit words, IEEE half)
 *     LBM_BF16S  bfloat16 f_i - w_i  (raw 16-bit words)
 *   Arithmetic runs in FP64 for LBM_F64 and in FP32 otherwise; every value written is
 *   rounded once to the storage format, to nearest even, subnormals kept.
 *
 * Real arrays (force, rho, u, adjoint populations, force gradients) use the "real"
 *   type of the storage kind: double for LBM_F64, float for every other kind.  Vector
 *   fields are SoA [D][N] (component a = x, y, z at offset a*N + n, n = (z*ny + y)*nx
 *   + x); adjoint population arrays use the population layout above.
 *
 * State: a population buffer holds the post-collision populations g(t) = C(f(t)) of
 *   Eq. 1's state f(t); one step maps g(t) to g(t+1) = C(S g(t)) where S is the
 *   periodic pull streaming (S g)_i(x) = g_i(x - c_i).  This is Eq. 1 regrouped so
 *   that one kernel reads each population once and writes it once.
 *
 * Memory and streams: every pointer argument is a device pointer owned by the caller
 *   (nothing is retained after a call returns), aligned to 16 bytes.  The library
 *   allocates no device memory.  `stream` is a hipStream_t (NULL = the null stream);
 *   all work is enqueued asynchronously on it and no call synchronises.
 *
 * Errors: every entry point validates its arguments on the host before any HIP call
 *   and returns a negative lbm_status without touching device memory when they are
 *   invalid.  A failed kernel launch returns LBM_EHIP; faults inside kernels surface at
 *   the caller's next synchronisation.  lbm_strerror()/lbm_last_error() describe codes.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum lbm_lattice { LBM_D2Q9 = 0, LBM_D3Q27 = 1, LBM_D3Q19 = 2 };

enum lbm_storage { LBM_F64 = 0, LBM_F32 = 1, LBM_F32S = 2, LBM_F16S = 3, LBM_BF16S = 4 };

enum lbm_status {
  LBM_OK = 0,
  LBM_EINVAL = -1, /* bad scalar argument: tau <= 1/2 or not finite, n_steps < 1,
                      dims < 1, nz != 1 for D2Q9, 0 < pitch < nx, unknown lattice or
                      storage, workspace too small */
  LBM_ENULL = -2,  /* a required pointer is NULL */
  LBM_EALIGN = -3, /* a pointer is not 16-byte aligned */
  LBM_EALIAS = -4, /* an output buffer overlaps an input buffer it must not overlap */
  LBM_EUNSUP = -5, /* unsupported combination of arguments */
  LBM_ERANGE = -6, /* grid too large: N > 2^31 - 1, a dimension > 2^31 - 1, or a row
                      of 4 GiB or more (pitch * real bytes >= 2^32, see Grid) */
  LBM_EHIP = -7    /* a HIP runtime call failed; lbm_last_error() has the text */
};

/* Grid descriptor.  lattice: enum lbm_lattice; storage: enum lbm_storage.
 * pitch: words between consecutive direction rows of a population buffer, 0 (= nx, no
 *   padding) or >= nx.  Population buffers (and adjoint population arrays) then hold
 *   Q*pitch*ny*nz words, word (i, x, y, z) at ((z*ny + y)*Q + i)*pitch + x.  The
 *   pitch - nx pad words of a direction row are never read.  lbm_step, lbm_step_shifted
 *   and lbm_step_slab may overwrite the pad words inside their rows' last block segment
 *   of 64, 128 or 256 cells with unspecified values (so that whole cache lines are
 *   written); every other entry point leaves pad words untouched, and
 *   lbm_slab_halo_copy moves them along with the face rows.  Rows whose byte length is
 *   a multiple of 256 (pitch a multiple of 64 for 4-byte words) keep the step near full
 *   bandwidth for any nx.  Real fields (rho, u, force) stay dense. */
typedef struct lbm_grid {
  int32_t lattice;
  int32_t storage;
  int64_t nx, ny, nz;
  int64_t pitch;
} lbm_grid;

/* Faces of a z-slab (lbm_slab_halo_copy). */
enum lbm_face { LBM_FACE_LOW = 0, LBM_FACE_HIGH = 1 };

/* Number of reduction results written by lbm_moments (see there). */
#define LBM_NRED 8

/* Static description of a status code (never NULL). */
const char* lbm_strerror(int status);

/* Text of the most recent failure on the calling thread (validation detail or HIP
 * error string); "" if none. */
const char* lbm_last_error(void);

/* Library ABI version (major*10000 + minor*100 + patch). */
int lbm_version(void);

/* Velocity set of a lattice (Sec. 2.1: c_i, w_i; the values are the textbook D2Q9,
 * D3Q19 and D3Q27 tables, the order is the library's).  Host pointers; any may be NULL.
 * D, Q: dimension and number of velocities.  c: Q*D ints, row i = (c_x, c_y[, c_z]).
 * w: Q doubles.  Returns LBM_OK or LBM_EINVAL for an unknown lattice. */
int lbm_lattice_info(int lattice, int* D, int* Q, int* c, double* w);

/* Writes the equilibrium populations f^eq(rho, u) (Eq. 3) of every cell into f_out,
 * which is then g(0): an equilibrium is a fixed point of the BGK collision, so it is
 * both the pre- and the post-collision state at t = 0.
 * rho: N doubles, or NULL for rho = 1 everywhere.  u: D*N doubles (SoA), required.
 * f_out: Q*N storage words.  f^eq is evaluated in FP64 and rounded once. */
int lbm_init_equilibrium(const lbm_grid* grid, const double* rho, const double* u,
                         void* f_out, void* stream);

/* Advances the populations by n_steps time steps g <- C(S g) (Eqs. 1-4), ping-ponging
 * between f_in and f_out: step k reads one buffer and writes the other, starting with
 * f_in -> f_out.  For n_steps > 1 both buffers are overwritten.
 * tau: BGK relaxation time (Eq. 2), tau > 1/2; the kinematic viscosity is
 *   nu = (tau - 1/2)/3 (Sec. 3.1).
 * force: D*N reals (SoA), or NULL for no force.  With a force the collision uses the
 *   Guo scheme: u = (sum c_i f_i + F/2)/rho in f^eq, plus the source
 *   (1 - 1/(2 tau)) w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F.
 * f_in and f_out must not overlap; force must not overlap either.
 * Returns 0 if the result is in f_out (odd n_steps), 1 if it is in f_in (even
 * n_steps), or a negative lbm_status.
 * Launches: where the grid allows it, several steps run as one launch of a kernel that
 * keeps the intermediate states on chip, so the state is read and written once per
 * launch: two steps on D3Q27 and D3Q19 (FP32 or shifted-FP32 words with nx a multiple
 * of 32 and ny of 8, shifted-FP16 or shifted-BF16 words with nx a multiple of 64 and
 * ny of 4, or FP64 words with nx a multiple of 32 and ny of 4; nz >= 3; one z plane of
 * words < 4 GiB), two or four on D2Q9 (every kind; nx a multiple of 64; ny >= 3 for
 * two, ny >= 5 for four; the 9 direction rows of a grid row < 4 GiB).  Results equal single
 * steps bit for bit.  Multi-step launches come in pairs of one kind (n_steps = 8 a + 4 b + c:
 * 2a launches of four steps, 2b of two, c < 4 single steps first), so the result stays
 * in the buffer named above.  Multi-step launches leave pad words untouched.
 * lbm_step_launches tells how a call is split. */
int lbm_step(const lbm_grid* grid, void* f_in, void* f_out, double tau, const void* force,
             int n_steps, void* stream);

/* How lbm_step (and lbm_step_shifted, and lbm_step_mrt) split
 * n_steps >= 1 into launches: *single
 * one-step launches, then *paired two-step launches, then *quad four-step launches
 * (single + 2 paired + 4 quad = n_steps; paired and quad are even).  Host-only (no
 * device work).  LBM_EINVAL for n_steps < 1, LBM_ENULL for NULL outputs, grid errors as
 * lbm_step. */
int lbm_step_launches(const lbm_grid* grid, int n_steps, int* single, int* paired, int* quad);

/* lbm_step with the flow-control forcing of Sec. 3.2 instead of a body force: the
 * equilibrium is evaluated at a locally shifted velocity, f^eq(rho, u + du), with
 * u = sum_i c_i f_i / rho (Eq. 4) and du a per-cell shift (D*N reals, required).
 * The collision then adds rho du / tau of momentum per cell and step.  Same ping-pong,
 * return value and argument rules as lbm_step. */
int lbm_step_shifted(const lbm_grid* grid, void* f_in, void* f_out, double tau, const void* du,
                     int n_steps, void* stream);

/* D2Q9 steps with the multiple-relaxation-time collision of Sec. 3.1 (Eq. 5),
 * Omega(f) = -M^{-1} S^{-1} (M f - m^eq), m^eq = M f^eq, in the Dellar moment basis
 * m = (rho, rho u, rho v, Pi_xx, Pi_xy, Pi_yy, N, J_x, J_y).
 * tau_moments: host array of 9 relaxation times S = diag(tau_0 .. tau_8); tau_0..2
 *   (conserved moments) are ignored, tau_3..8 must be finite and > 1/2.  The shear
 *   times tau_3..5 set nu = (tau - 1/2)/3; all nine equal give BGK.
 * tau_ghost: NULL, or 3*N reals giving per-cell tau_6, tau_7, tau_8 (N, J_x, J_y) in
 *   place of the uniform ones (the outputs of the paper's neural collision model);
 *   every value must be > 1/2 (not checked on the device).
 * Same ping-pong, return value and buffer rules as lbm_step.  With uniform ghost times
 * or a tau_ghost field the steps run two or four per launch where lbm_step's would
 * (lbm_step_launches; the field is read a row ahead, as a force), bit for bit the
 * single steps.  LBM_EUNSUP for lattices other than D2Q9. */
int lbm_step_mrt(const lbm_grid* grid, void* f_in, void* f_out, const double* tau_moments,
                 const void* tau_ghost, int n_steps, void* stream);

/* One step (Eqs. 1-4, as lbm_step) on a z-slab: one shard of a grid that is periodic
 * in x and y and split into slabs of consecutive planes along z, each slab stepping
 * on its own device with ghost planes for the populations that cross its faces.
 * slab: D3Q19 or D3Q27 (LBM_EUNSUP otherwise); nx, ny as the whole grid, nz = the
 *   slab's own planes.
 * f_in, f_out: slab buffers of (nz + 2) planes in the population layout, i.e. the
 *   layout of a grid of nz + 2 planes: buffer plane 0 is the ghost plane below the
 *   slab, planes 1..nz hold slab planes 0..nz-1, plane nz + 1 is the ghost plane
 *   above.  The pull gather of slab plane 0 reads the directions with c_z = +1 from
 *   the lower ghost plane, that of plane nz-1 the directions with c_z = -1 from the
 *   upper one (filled by lbm_slab_halo_copy); no other ghost words are read, and
 *   nothing wraps in z.
 * z_begin, z_end: the slab planes [z_begin, z_end) to compute, 0 <= z_begin < z_end
 *   <= nz; only those planes of f_out are written.  Splitting a step into the inner
 *   planes [1, nz-1), which need no ghost data, and the two boundary planes lets the
 *   halo exchange of the previous step overlap the inner work.
 * tau, force: as in lbm_step; force holds D*nx*ny*nz reals for the slab's own cells.
 * f_in and f_out must not overlap; force must not overlap either.  Returns LBM_OK. */
int lbm_step_slab(const lbm_grid* slab, const void* f_in, void* f_out, double tau,
                  const void* force, int64_t z_begin, int64_t z_end, void* stream);

/* Halo exchange of the slab step: copies the populations that leave a slab through one
 * face into the ghost plane of the neighbouring slab on that side (Eq. 1's streaming
 * across the cut).
 *   LBM_FACE_LOW:  directions with c_z = -1 of src's lowest plane (buffer plane 1)
 *                  into dst's upper ghost plane (buffer plane nz_dst + 1);
 *   LBM_FACE_HIGH: directions with c_z = +1 of src's highest plane (buffer plane
 *                  nz_src) into dst's lower ghost plane (buffer plane 0).
 * Those directions are consecutive in the velocity order (9 of 27, 5 of 19), so each
 * grid row moves one contiguous run of n_dir*nx words.  The two slabs must agree in
 * lattice, storage, nx and ny (nz may differ); src and dst may be the same buffer (one
 * slab that is its own periodic neighbour) but the source plane must not overlap the
 * destination ghost plane. */
int lbm_slab_halo_copy(const lbm_grid* src_slab, const void* src, const lbm_grid* dst_slab,
                       void* dst, int face, void* stream);

/* Two steps (Eqs. 1-4, as lbm_step with n_steps = 2) of a whole z-slab in one launch
 * that keeps the intermediate state on chip, for slabs with two ghost planes on each
 * side: the halo of two steps is two planes deep, so the slabs exchange once per two
 * steps.
 * slab: as lbm_step_slab, nz >= 2 (LBM_EINVAL otherwise, and for an empty or
 *   out-of-range plane range).
 * f_in, f_out: slab buffers of (nz + 4) planes in the population layout: buffer
 *   planes 0 and 1 are the ghost planes -2 and -1 below the slab, planes 2 .. nz + 1 hold
 *   slab planes 0 .. nz-1, planes nz + 2 and nz + 3 the ghost planes nz and nz + 1
 *   above.  The intermediate step is computed on planes -1 .. nz, which reads the
 *   directions with c_z = +1 of ghost plane -2, those with c_z = 0 and +1 of ghost plane
 *   -1, those with c_z = 0 and -1 of ghost plane nz and those with c_z = -1 of ghost plane
 *   nz + 1 (what lbm_slab2_halo_copy fills); no other ghost words are read.  The ghost
 *   planes of f_out are left alone.
 * force: NULL, or D * nx * ny * (nz + 2) reals: the force of slab planes -1 .. nz (one
 *   ghost plane each side, which the caller fills from the neighbours' force).
 * z_begin, z_end: the slab planes [z_begin, z_end) to compute, 0 <= z_begin < z_end
 *   <= nz; only those planes of f_out are written.  The inner planes [2, nz-2) read no
 *   ghost data, so they can run while the halo exchange of the previous launch is in
 *   flight, and the four boundary planes after it.
 * The result equals two steps of the periodic grid the slabs make up bit for bit.
 * LBM_EUNSUP where the slab or storage kind does not take the two-step kernel (3D
 * lattices; nx and ny on lbm_step's two-step tiles; lbm_step_slab2_available).  f_in and
 * f_out must not overlap, nor force either of them. */
int lbm_step_slab2(const lbm_grid* slab, const void* f_in, void* f_out, double tau, const void* force,
                   int64_t z_begin, int64_t z_end, void* stream);

/* *available = 1 if lbm_step_slab2 takes this slab and storage kind, else 0.
 * Host-only.  Grid errors as lbm_step; LBM_ENULL for a NULL output. */
int lbm_step_slab2_available(const lbm_grid* slab, int* available);

/* Halo exchange of lbm_step_slab2 (Eq. 1's streaming across the cut, two planes deep):
 *   LBM_FACE_LOW:  src's slab plane 0, directions with c_z = -1 and 0, into dst's ghost
 *                  plane nz_dst, and src's plane 1, c_z = -1, into dst's ghost plane
 *                  nz_dst + 1 (dst is the slab below src);
 *   LBM_FACE_HIGH: src's plane nz_src - 1, c_z = 0 and +1, into dst's ghost plane -1,
 *                  and src's plane nz_src - 2, c_z = +1, into dst's ghost plane -2 (dst is
 *                  the slab above).
 * Buffers of (nz + 4) planes as lbm_step_slab2; both slabs nz >= 2; other rules as
 * lbm_slab_halo_copy. */
int lbm_slab2_halo_copy(const lbm_grid* src_slab, const void* src, const lbm_grid* dst_slab, void* dst,
                        int face, void* stream);

/* Activation of the neural collision's hidden layer (lbm_step_neural). */
enum lbm_activation { LBM_ACT_RELU = 0, LBM_ACT_TANH = 1 };

/* Number of parameters of the neural collision's network. */
#define LBM_NEURAL_PARAMS 530

/* D2Q9 steps with the neural collision model of Sec. 3.1: the MRT collision of Eq. 5
 * (as lbm_step_mrt) with tau_0..2 = 1, tau_3..5 = tau_shear, and tau_6, tau_7, tau_8
 * given per cell and step by a shallow network, tau_n = exp(t_n) + 1/2.
 * The paper fixes one hidden layer, 530 parameters, local moments as inputs and the
 * exp(.) + 1/2 output map; the library reads it as
 *   inputs  x = (Pi_xx, Pi_xy, Pi_yy, N, J_x, J_y) of the non-equilibrium part h - f^eq
 *           of the streamed populations (Dellar's rows c_x^2, c_x c_y, c_y^2, g, g c_x,
 *           g c_y, g = (3c_x^2-1)(3c_y^2-1));
 *   hidden  a_j = act(b1_j + sum_k W1_jk x_k), j = 0..52;
 *   output  t_n = sum_j W2_nj a_j, n = 0..2 (tau_6, tau_7, tau_8), no output bias;
 * 6*53 + 53 + 3*53 = 530 parameters.
 * params: LBM_NEURAL_PARAMS reals (device) in the order W1 [53][6] row-major, b1 [53],
 *   W2 [3][53] row-major; arithmetic in the storage kind's real type.
 * activation: LBM_ACT_RELU or LBM_ACT_TANH.
 * tau_shear > 1/2 sets nu = (tau_shear - 1/2)/3.  Same ping-pong, return value and
 * buffer rules as lbm_step (one step per launch); params must not overlap the population
 * buffers.  LBM_EUNSUP for lattices other than D2Q9. */
int lbm_step_neural(const lbm_grid* grid, void* f_in, void* f_out, double tau_shear,
                    const void* params, int activation, int n_steps, void* stream);

/* Streaming only: f_out_i(x) = f_in_i(x - c_i), periodic (Eq. 1's shift), copying the
 * raw storage words (a permutation: bit-exact for every storage kind).  Buffers must not
 * overlap. */
int lbm_stream_only(const lbm_grid* grid, const void* f_in, void* f_out, void* stream);

/* Plain device-to-device copy of `bytes` (a multiple of 16) with one 16-byte word per
 * thread, nontemporal loads and stores: the practical HBM bandwidth reference that the
 * step kernel's GB/s are compared with (no part of the method).  Buffers must not
 * overlap. */
int lbm_copy(const void* src, void* dst, size_t bytes, void* stream);

/* Bytes of device workspace lbm_moments needs when it computes reductions. */
int lbm_moments_workspace_size(const lbm_grid* grid, size_t* bytes);

/* Macroscopic fields of the state g (Eq. 4) and FP64 reductions over the grid.
 * rho_out: N reals or NULL.  u_out: D*N reals or NULL.
 *   rho = sum_i g_i; u = (sum_i c_i g_i - F/2)/rho, i.e. the density and the (Guo)
 *   velocity of the pre-collision state f(t) whose collision produced g(t).
 * force: D*N reals or NULL (must match what the steps used).
 * red: NULL, or a device array of LBM_NRED doubles receiving, in FP64:
 *   [0] sum rho   [1..3] sum rho u_a (z = 0 in 2D)   [4] kinetic energy 1/2 sum |u|^2
 *   [5] number of cells whose rho or u is not finite   [6] max |u|   [7] min rho
 *   The reduction order depends only on the grid and on whether a field is written,
 *   so repeated calls are bitwise reproducible.  A call that writes rho_out or u_out
 *   sums [0..4] in another order than one that writes neither: the two agree to FP64
 *   rounding, and [5..7], which do not depend on the order, agree exactly.
 * workspace: device scratch of lbm_moments_workspace_size() bytes, required iff red is
 *   not NULL; its contents are clobbered. */
int lbm_moments(const lbm_grid* grid, const void* g, const void* force, void* rho_out,
                void* u_out, double* red, void* workspace, size_t workspace_bytes,
                void* stream);

/* lbm_moments without a workspace argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments, results and errors as lbm_moments with the workspace
 * left out: the fields and the reductions are bitwise those of lbm_moments on the same
 * inputs.  The reduction partials go to a fixed 8 MiB device array inside the library
 * (131072 partials of LBM_NRED doubles), one per GPU, set up on the first call on that
 * GPU and held until the process ends; the call allocates nothing and frees nothing.
 * Grids whose reduction needs more partials than that return LBM_ERANGE (use
 * lbm_moments): with red != NULL, the partials are one per 256 cells (3D lattices
 * writing rho_out or u_out: up to about 33.5 million cells), per 1024 cells (D2Q9
 * writing fields: about 134 million) or per 4096 cells (no field written: about 536
 * million), plus one per 2048 partials.  Every call on a GPU shares that GPU's array and
 * overwrites what it needs before reading it (nothing has to start at zero), so calls
 * that overlap on one GPU (on different streams without ordering, or from several
 * threads) race and give wrong reductions.  The first call on a GPU may return LBM_EHIP
 * if the array's address cannot be obtained. */
int lbm_moments_noalloc(const lbm_grid* grid, const void* g, const void* force, void* rho_out, void* u_out,
                        double* red, void* stream);

/* Reverse-mode derivative of one lbm_step (hand-written adjoint; the paper obtains the
 * same quantity by automatic differentiation, Sec. 3.2).  With g' = C(S g_t; F):
 *   lam_out = (dg'/dg_t)^T lam_next          (overwritten, Q*N reals)
 *   dforce += (dg'/dF)^T lam_next            (accumulated, D*N reals; may be NULL)
 * g_t: the state the forward step started from (storage words).  lam_next: Q*N reals,
 * dL/dg(t+1).  For shifted storage the derivative is taken with respect to f_i (equal to
 * the one with respect to f_i - w_i); rounding to storage is not differentiated.
 * tau and force as in lbm_step; dforce requires force.  lam_out must not overlap g_t,
 * lam_next, force or dforce. */
int lbm_adjoint_step(const lbm_grid* grid, const void* g_t, const void* lam_next, void* lam_out,
                     double tau, const void* force, void* dforce, void* stream);

/* The adjoint step of lbm_adjoint_step in its collision-local form, the one the
 * checkpointed rollout runs (derivatives of the step as in Sec. 3.2).  The streaming is
 * moved out of the step's transpose, so every write is aligned: with lam_{t+1} =
 * adj_next (adj_is_chi = 0) or lam_{t+1} = S^T adj_next (adj_is_chi = 1: adj_next holds
 * chi_{t+1}, read gathered as chi_{t+1,i}(x + c_i)),
 *   chi_out = J_C(S g_t)^T lam_{t+1}       (overwritten, Q*N reals, aligned with g_t)
 *   dforce += (dg'/dF)^T lam_{t+1}         (accumulated, D*N reals; may be NULL)
 * and lam_t = S^T chi_t (lbm_adjoint_unstream).  adj_is_chi must be 0 or 1 (LBM_EINVAL
 * otherwise).  Layout, tau, force, dforce, aliasing rules and errors as lbm_adjoint_step. */
int lbm_adjoint_step_local(const lbm_grid* grid, const void* g_t, const void* adj_next, int adj_is_chi,
                           void* chi_out, double tau, const void* force, void* dforce, void* stream);

/* Two steps of lbm_adjoint_step_local with chi in and chi out, in one launch that keeps
 * the intermediate chi on chip (derivatives of the step as in Sec. 3.2; two steps of
 * the rollout's backward pass):
 *   chi_out = J_C(S g_tm1)^T S^T [ J_C(S g_t)^T S^T chi_next ]
 *   dforce += the two steps' contributions, added in the order of two calls (step t
 *             first), so that the result equals lbm_adjoint_step_local(g_t, chi_next,
 *             1, tmp) followed by lbm_adjoint_step_local(g_tm1, tmp, 1, chi_out) bit for
 *             bit.
 * g_t, g_tm1: the states of steps t and t-1 (Q*N storage words each, read only).
 * chi_next: Q*N reals (read only).  chi_out: Q*N reals, live cells overwritten, pad
 * words untouched.  tau, force, dforce as lbm_adjoint_step (the one force field of both
 * steps).  LBM_EALIAS if chi_out or dforce overlaps another argument.  LBM_EUNSUP for
 * dforce without force, and where the grid or storage kind is not taken: the kernel
 * takes D3Q27 and D3Q19 grids with any storage kind but FP64, nx a multiple of 32, ny
 * of 8, nz >= 3 and one z plane of reals < 4 GiB (lbm_adjoint_step2_available). */
int lbm_adjoint_step2_local(const lbm_grid* grid, const void* g_t, const void* g_tm1, const void* chi_next,
                            void* chi_out, double tau, const void* force, void* dforce, void* stream);

/* *available = 1 if lbm_adjoint_step2_local takes this grid and storage kind, else 0.
 * Host-only.  Grid errors as lbm_step; LBM_ENULL for a NULL output. */
int lbm_adjoint_step2_available(const lbm_grid* grid, int* available);

/* lam_out = S^T chi, the transpose of the pull streaming of Eq. 1: lam_out_i(x) =
 * chi_i(x + c_i) with periodic wrap, on Q*N reals in the population layout (FP64 for
 * FP64 storage, FP32 otherwise).  Turns the local form's chi into lam.  chi and lam_out
 * are caller-owned device buffers and must not overlap (LBM_EALIAS). */
int lbm_adjoint_unstream(const lbm_grid* grid, const void* chi, void* lam_out, void* stream);

/* Reverse-mode derivative of lbm_moments' fields (Eq. 4's moments, rho = sum_i g_i and
 * rho u = sum_i c_i g_i - F/2; the terminal step of the automatic differentiation of
 * Sec. 3.2, where the cost is a function of the velocity field): with
 * (rho, u) = moments(g; F),
 *   lam_out = (drho/dg)^T dL_drho + (du/dg)^T dL_du       (overwritten, Q*N reals)
 *   dforce += (du/dF)^T dL_du = -dL_du / (2 rho)           (accumulated, may be NULL)
 * i.e. lam_out_i = dL_drho + (c_i - u).dL_du / rho per cell.
 * dL_drho: N reals or NULL (zero); dL_du: D*N reals or NULL (zero), in the real type
 * and SoA layout above.  g is read, lam_out written in the population layout.  lam_out
 * and dforce must not overlap any other argument (LBM_EALIAS); dforce needs force
 * (LBM_EUNSUP).  Errors as lbm_moments. */
int lbm_moments_adjoint(const lbm_grid* grid, const void* g, const void* force,
                        const void* dL_drho, const void* dL_du, void* lam_out, void* dforce,
                        void* stream);

/* ---- Loss head of the flow-control forcing (Sec. 3.2) ----------------------------
 * The paper steers a decaying flow by a cost on its instantaneous energy spectrum; the
 * controlled step needs that cost's gradient every step.  With uh_a(k) the
 * unnormalised forward FFT of the velocity component u_a (taken by the caller), s =
 * 1/N and shells K = floor(|k| + 1/2) of the integer wavevectors k:
 *   E(K) = s^2/2 sum_{k in K} sum_a |uh_a(k)|^2          (shell energy spectrum)
 *   R    = sum_{K=k_lo..k_hi} (ln max(E_K, c) - ln max(Et_K, c))^2
 *   dR/du_a = Re IFFT(g s uh_a), g(k) = dR/dE_K at the shell of k
 * (IFFT normalised by 1/N), so a step is: FFT, lbm_shell_energy,
 * lbm_log_spectrum_grad, inverse FFT, lbm_real_part (-> the du of lbm_step_shifted).
 *
 * lbm_shells describes the wavevectors grouped by shell, all device arrays owned by the
 * caller: order[n] the flat wavevector indices sorted by shell, offsets[nshell + 1]
 * with shell K = order[offsets[K] .. offsets[K+1]) (offsets[0] = 0, offsets[nshell] =
 * n), shell[n] the shell of every flat wavevector.  A table that breaks these rules
 * gives wrong results but no access outside the arrays.  1 <= n <= 2^31 - 1 and
 * nshell >= 1 (LBM_EINVAL / LBM_ERANGE otherwise). */
typedef struct {
  int64_t n;
  int32_t nshell;
  const int32_t* order;
  const int32_t* offsets;
  const int32_t* shell;
} lbm_shells;

/* E[0 .. nshell) <- s^2/2 sum over each shell of sum_a |uhat_a(k)|^2, deterministic
 * (fixed summation order).  uhat: D*n complex doubles (interleaved re, im), component
 * a at uhat[a*n + k]; D in 1..3.  scale = s.  E must not overlap uhat or the shell
 * table (LBM_EALIAS). */
int lbm_shell_energy(const lbm_shells* shells, int D, const void* uhat, double scale, double* E, void* stream);

/* uhat_a(k) *= scale * dR/dE_K (in place; K the shell of k): 2 (ln E_K - ln max(Et_K, c))
 * / E_K for k_lo <= K <= k_hi and E_K >= c, else 0.  E, E_target: nshell doubles.  R: one
 * double receiving R, or NULL.  0 <= k_lo <= k_hi < nshell and a finite cutoff c > 0
 * (LBM_EINVAL otherwise); uhat and R must not overlap each other, E, E_target or the
 * shell table (LBM_EALIAS). */
int lbm_log_spectrum_grad(const lbm_shells* shells, int D, void* uhat, const double* E, const double* E_target,
                          int k_lo, int k_hi, double cutoff, double scale, double* R, void* stream);

/* out[i] = scale * Re z[i], i < count: z complex doubles, out FP32 (out_storage LBM_F32)
 * or FP64 (LBM_F64); they must not overlap. */
int lbm_real_part(const void* z, int64_t count, double scale, void* out, int out_storage, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */

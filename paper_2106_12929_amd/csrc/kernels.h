// Internal interface between the C ABI layer (api.hip) and the kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int kNred = 8;              // reduction results of lbm_moments
enum AdjointMode { kAdjScatter = 0, kAdjLocalLam = 1, kAdjLocalChi = 2 };
enum ForceMode { kNoForce = 0, kGuoForce = 1, kShiftForce = 2 };
// Collisions of the D2Q9 multi-step kernel in place of BGK (its force-mode parameter):
// the MRT collision, unforced, with uniform relaxation times or with per-cell ghost
// times read from a field (tau_6, tau_7, tau_8 at a stride of the cell count).
constexpr int kMrtUniform = 3;
constexpr int kMrtField = 4;
constexpr int kFoldBlock = 2048;  // block partials folded by one block of the second reduction stage

// Grid geometry passed by value to every cell-parallel kernel.
struct GridArgs {
  uint32_t nx, ny, nz;
  uint32_t block_x;  // cells of one row handled by a 256-thread block: 64, 128 or 256
  uint64_t ncells;   // nx * ny * nz (< 2^31)
  uint32_t z0, nzl;  // planes [z0, z0 + nzl) handled by the launch (0 and nz: all of them)
  uint32_t ghost;    // 0: periodic in z; 1: z-slab buffer with a ghost plane below and above
                     // the nz planes (buffer plane = z + 1, no wrap in z); 2: two ghost
                     // planes each side (buffer plane = z + 2), step2_kernel only
  uint32_t pitch;    // words between direction rows of population buffers (>= nx)
};

hipError_t launch_step(int lattice, int storage, const void* fin, void* fout, const void* force, int force_mode,
                       const GridArgs& g, double omega, hipStream_t s);

// Launch geometry of the two-step kernel (step2_kernel).
struct Step2Args {
  uint32_t tiles_x, tiles_y;  // tiles of the grid's (x, y) columns
  uint32_t lz;                // planes per z chunk (the last chunk may be shorter)
  uint32_t row_bytes;         // one direction row: pitch words
  uint32_t yrow_bytes;        // the Q direction rows of one grid row
  uint32_t plane_bytes;       // the ny grid rows of one z plane (< 2^32)
  uint64_t force_stride;      // reals between the force components (the force field's cells)
};
// The most steps one launch can advance for this lattice, storage kind and grid: 4
// (the D2Q9 multi-step kernel), 2 (the two-step kernels) or 1.  For nst = 2 or 4 up to
// that, launch_stepn(fin -> fout) equals nst launches of launch_step bit for bit.
int max_steps_per_launch(int lattice, int storage, const GridArgs& g);
hipError_t launch_stepn(int lattice, int storage, int nst, const void* fin, void* fout, const void* force,
                        int force_mode, const GridArgs& g, double omega, hipStream_t s);
// nst = 2 or 4 steps of the D2Q9 MRT collision in one launch (stepn_2d_kernel), where
// launch_stepn would take the grid; scales as launch_mrt; ghost: NULL for uniform
// relaxation times, else the per-cell ghost-time field.
hipError_t launch_stepn_mrt(int storage, int nst, const void* fin, void* fout, const GridArgs& g,
                            const double* scales, const void* ghost, hipStream_t s);
hipError_t launch_stream(int lattice, int word_bytes, const void* fin, void* fout, const GridArgs& g, hipStream_t s);
hipError_t launch_init(int lattice, int storage, const double* rho, const double* u, void* fout, const GridArgs& g,
                       hipStream_t s);
// Entries (kNred doubles each) of the workspace of launch_moments with reductions: at most
// one partial per block of the one-thread-per-cell launch, then one per kFoldBlock of
// those.
uint64_t moments_workspace_entries(const GridArgs& g);
// Entries the reducing launch for this lattice actually uses (its span depends on the
// lattice and on whether fields are written): at most moments_workspace_entries.
uint64_t moments_entries_used(int lattice, const GridArgs& g, bool fields);
hipError_t launch_moments(int lattice, int storage, const void* f, const void* force, void* rho, void* u,
                          double* workspace, double* red, const GridArgs& g, hipStream_t s);
hipError_t launch_adjoint(int lattice, int storage, int mode, const void* gt, const void* lam_next, void* lam_out,
                          const void* force, void* dforce, const GridArgs& g, double omega, hipStream_t s);
// Two collision-local adjoint steps, chi_next -> chi_out through g_t and g_t-1
// (adjoint2_kernel), where the grid and storage kind allow; equal to two launch_adjoint
// calls in mode kAdjLocalChi bit for bit, the force gradient included.
bool adjoint2_supported(int lattice, int storage, const GridArgs& g);
// Two steps on a z-slab with two ghost planes on each side (step2_kernel with
// g.ghost == 2): buffer plane p + 2 holds slab plane p (p = -2 .. nz + 1), the force
// holds slab planes -1 .. nz at p + 1.  Planes [g.z0, g.z0 + g.nzl) are computed;
// nothing wraps in z.
bool step2_slab_supported(int lattice, int storage, const GridArgs& g);
hipError_t launch_step2_slab(int lattice, int storage, const void* fin, void* fout, const void* force,
                             int force_mode, const GridArgs& g, double omega, hipStream_t s);
hipError_t launch_adjoint2(int lattice, int storage, const void* gt, const void* gtm1, const void* chi_next,
                           void* chi_out, const void* force, void* dforce, const GridArgs& g, double omega,
                           hipStream_t s);
hipError_t launch_unstream(int lattice, int word_bytes, const void* fin, void* fout, const GridArgs& g,
                           hipStream_t s);
// Source of the MRT ghost times tau_6..8 (see mrt_step_kernel).
enum GhostMode { kGhostUniform = 0, kGhostField = 1, kGhostRelu = 2, kGhostTanh = 3 };
constexpr int kNeuralHidden = 53;                            // hidden units of the neural collision
constexpr int kNeuralParams = 6 * kNeuralHidden + kNeuralHidden + 3 * kNeuralHidden;  // 530
// scales[k] = 1 / (tau_{k+3} |R_{k+3}|^2), k = 0..5 (see mrt_step_kernel); ghost: the
// per-cell times (kGhostField) or the network parameters (kGhostRelu, kGhostTanh).
hipError_t launch_mrt(int storage, const void* fin, void* fout, const void* ghost, int ghost_mode, const GridArgs& g,
                      const double* scales, hipStream_t s);
// Copies n_dir consecutive direction rows (of `pitch` words) of every grid row of plane
// `src_plane` of src into plane `dst_plane` of dst (planes in buffer coordinates),
// starting at direction i0: the face populations of a z-slab halo exchange.
hipError_t launch_halo_copy(int Q, int word_bytes, const void* src, uint64_t src_plane, void* dst, uint64_t dst_plane,
                            int i0, int n_dir, uint32_t pitch, uint32_t ny, hipStream_t s);
hipError_t launch_copy16(const void* src, void* dst, size_t n16, hipStream_t s);
hipError_t launch_moments_adjoint(int lattice, int storage, const void* f, const void* force, const void* drho,
                                  const void* du, void* lam_out, void* dforce, const GridArgs& g, hipStream_t s);

// Loss head of the flow-control forcing (spectrum.hip).
hipError_t launch_shell_energy(const void* uh, int D, uint32_t n, const int32_t* order, const int32_t* offsets,
                               int nshell, double scale, double* E, hipStream_t s);
hipError_t launch_log_spectrum_grad(void* uh, int D, uint32_t n, const int32_t* shell, const double* E,
                                    const double* Et, int nshell, int k_lo, int k_hi, double cutoff, double scale,
                                    double* R, hipStream_t s);
hipError_t launch_real_part(const void* z, uint64_t count, double scale, void* out, bool f64, hipStream_t s);

}  // namespace lbm

// LDS-staged fused stream + BGK collide (Eqs. 1-4) for 2- and 4-byte storage words.
//
// Same arithmetic, launch grid and results as step_kernel (kernels.hip); only the way
// the words move differs.  A block handles a segment of BX cells in each of 256/BX
// consecutive rows, and every global access is a 16-byte vector:
//   1. stage: for each of the 9 source rows (y - c_y, z - c_z) of a row, the directions
//      with that (c_y, c_z) are consecutive direction rows in memory (c_x varies
//      fastest in the velocity order).  Their segment [x0 - V, x0 + BX + V) (V words
//      per vector, periodic in x) is loaded with nontemporal 16-byte loads into LDS;
//   2. collide: each thread gathers its Q pull-streamed words from LDS (the +-1 shift
//      in x is an LDS offset), runs bgk_collide and writes the results back into LDS;
//   3. store: the block writes its Q output segments with nontemporal 16-byte stores.
// Requirements (checked by the launcher): nx is a multiple of BX (so no block segment
// is ragged and every vector index needs at most one periodic wrap) and the word is at
// most 4 bytes (FP64 rows would need 55 KB of LDS per block, too few blocks per CU).
// On the 256^3 D3Q27 FP32 grid the 16-byte streams lift the step from about 5.8 to
// 6.1 TB/s over the one-word-per-lane kernel, with identical output bits.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"
#include "kernels.h"
#include "lattice.h"

namespace lbm {

namespace {

// Source piece p = 3 (c_z + 1) + (c_y + 1): its first direction and its number of
// directions (3 for D3Q27 and D2Q9 pieces, 1 or 3 for D3Q19, 0 if absent).
template <typename LT>
__host__ __device__ constexpr int piece_first(int p) {
  for (int i = 0; i < LT::Q; ++i)
    if (3 * (LT::cz(i) + 1) + LT::cy(i) + 1 == p) return i;
  return 0;
}
template <typename LT>
__host__ __device__ constexpr int piece_size(int p) {
  int n = 0;
  for (int i = 0; i < LT::Q; ++i)
    if (3 * (LT::cz(i) + 1) + LT::cy(i) + 1 == p) ++n;
  return n;
}

template <int L, int S, int FM, int BX>
__global__ __launch_bounds__(256) void step_lds_kernel(const typename Storage<S>::word* __restrict__ fin,
                                                       typename Storage<S>::word* __restrict__ fout,
                                                       const typename Storage<S>::real* __restrict__ force,
                                                       GridArgs g, typename Storage<S>::real omega) {
  using LT = Lattice<L>;
  using ST = Storage<S>;
  using W = typename ST::word;
  using real = typename ST::real;
  using CO = Coef<L, real>;
  constexpr int Q = LT::Q;
  constexpr uint32_t V = 16 / sizeof(W);  // words per 16-byte vector
  constexpr uint32_t RB = 256 / BX;       // rows per block
  constexpr uint32_t P = BX / V + 2;      // vectors staged per direction: segment + one each side
  constexpr uint32_t VB = BX / V;         // vectors written per direction
  static_assert(sizeof(W) <= 4 && BX % V == 0, "LDS staging needs 2- or 4-byte words");
  __shared__ u32x4 stage[RB * Q * P];
  W* sw = reinterpret_cast<W*>(stage);

  const uint32_t blocks_x = g.nx / BX;
  const uint32_t bxi = blockIdx.x % blocks_x;
  const uint32_t row0 = (blockIdx.x / blocks_x) * RB;
  const uint32_t rows = g.ny * g.nzl;
  const uint32_t nv = g.nx / V;  // vectors per direction row
  const int32_t jb = (int32_t)(bxi * VB) - 1;
  const u32x4* __restrict__ vin = reinterpret_cast<const u32x4*>(fin);
  u32x4* __restrict__ vout = reinterpret_cast<u32x4*>(fout);

  // 1. Stage the source segments.  Stage slot s of direction i of row rb holds the word
  //    at x = x0 - V + s (periodic).
#pragma unroll
  for (uint32_t rb = 0; rb < RB; ++rb) {
    const uint32_t r = row0 + rb;
    if (r >= rows) break;
    const uint32_t y = r % g.ny, z = g.z0 + r / g.ny;
    // index c + 1 holds the coordinate of x - c (c = -1, 0, 1), as in sources()
    const uint32_t ys[3] = {wrap_inc(y, g.ny), y, wrap_dec(y, g.ny)};
    uint32_t zs[3];
    if (g.ghost) {
      zs[0] = z + 2;
      zs[1] = z + 1;
      zs[2] = z;
    } else {
      zs[0] = wrap_inc(z, g.nz);
      zs[1] = z;
      zs[2] = wrap_dec(z, g.nz);
    }
#pragma unroll
    for (int p = 0; p < 9; ++p) {
      const int n = piece_size<LT>(p);
      if (n == 0) continue;
      const int i0 = piece_first<LT>(p);
      const int cy = p % 3 - 1, cz = p / 3 - 1;
      const uint64_t src_row = ((uint64_t)zs[cz + 1] * g.ny + ys[cy + 1]) * Q + (uint64_t)i0;
      for (uint32_t k = threadIdx.x; k < (uint32_t)n * P; k += 256) {
        const uint32_t dir = k / P, jj = k - dir * P;
        int32_t j = jb + (int32_t)jj;
        j += j < 0 ? (int32_t)nv : 0;
        j -= j >= (int32_t)nv ? (int32_t)nv : 0;
        stage[(rb * Q + (uint32_t)i0 + dir) * P + jj] =
            __builtin_nontemporal_load(&vin[(src_row + dir) * nv + (uint32_t)j]);
      }
    }
  }
  __syncthreads();

  // 2. Collide.  Waves never straddle rows (BX is a multiple of 64).
  const uint32_t ty = __builtin_amdgcn_readfirstlane(threadIdx.x / BX);
  const uint32_t lx = threadIdx.x % BX;
  const uint32_t r = row0 + ty;
  const bool live = r < rows;
  // The words to store are formed right after the collision, in the same basic block as
  // its last arithmetic, so the compiler rounds to the storage format exactly as in
  // step_kernel (for 16-bit words it fuses the last FMA with the conversion) and both
  // kernels give identical bits.
  W out[Q];
  if (live) {
    const uint32_t base = ty * Q * P * V + V + lx;
    real d[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) d[i] = ST::to_dev(sw[base + (uint32_t)i * P * V - LT::cx(i)], CO::W(i));
    real Fx = 0, Fy = 0, Fz = 0;
    if constexpr (FM != kNoForce) {
      const size_t N = g.ncells;
      const uint32_t y = r % g.ny, z = g.z0 + r / g.ny;
      const uint32_t self = (z * g.ny + y) * g.nx + bxi * BX + lx;
      Fx = force[self];
      Fy = force[N + self];
      if constexpr (LT::D == 3) Fz = force[2 * N + self];
    }
    bgk_collide<L, real, FM>(d, Fx, Fy, Fz, omega);
#pragma unroll
    for (int i = 0; i < Q; ++i) out[i] = ST::from_dev(d[i], CO::W(i));
  }
  __syncthreads();
  if (live) {
    const uint32_t base = ty * Q * P * V + V + lx;
#pragma unroll
    for (int i = 0; i < Q; ++i) sw[base + (uint32_t)i * P * V] = out[i];
  }
  __syncthreads();

  // 3. Store the output segments (vectors 1 .. VB of each staged direction).
#pragma unroll
  for (uint32_t rb = 0; rb < RB; ++rb) {
    const uint32_t rr = row0 + rb;
    if (rr >= rows) break;
    const uint32_t y = rr % g.ny, zo = g.z0 + rr / g.ny + g.ghost;
    const uint64_t out_row = ((uint64_t)zo * g.ny + y) * Q;
    for (uint32_t k = threadIdx.x; k < (uint32_t)Q * VB; k += 256) {
      const uint32_t i = k / VB, jj = k % VB;
      __builtin_nontemporal_store(stage[(rb * Q + i) * P + 1 + jj], &vout[(out_row + i) * nv + bxi * VB + jj]);
    }
  }
}

template <int L, int S, int FM>
hipError_t launch_bx(const void* fin, void* fout, const void* force, const GridArgs& g, double omega, dim3 grid,
                     hipStream_t s) {
  using ST = Storage<S>;
  using W = typename ST::word;
  using R = typename ST::real;
  switch (g.block_x) {
    case 64:
      step_lds_kernel<L, S, FM, 64><<<grid, 256, 0, s>>>((const W*)fin, (W*)fout, (const R*)force, g, (R)omega);
      break;
    case 128:
      step_lds_kernel<L, S, FM, 128><<<grid, 256, 0, s>>>((const W*)fin, (W*)fout, (const R*)force, g, (R)omega);
      break;
    case 256:
      step_lds_kernel<L, S, FM, 256><<<grid, 256, 0, s>>>((const W*)fin, (W*)fout, (const R*)force, g, (R)omega);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int L, int S>
hipError_t launch_ls(const void* fin, void* fout, const void* force, int force_mode, const GridArgs& g, double omega,
                     dim3 grid, hipStream_t s) {
  if (!force || force_mode == kNoForce) return launch_bx<L, S, kNoForce>(fin, fout, nullptr, g, omega, grid, s);
  if (force_mode == kGuoForce) return launch_bx<L, S, kGuoForce>(fin, fout, force, g, omega, grid, s);
  if (force_mode == kShiftForce) return launch_bx<L, S, kShiftForce>(fin, fout, force, g, omega, grid, s);
  return hipErrorInvalidValue;
}

template <int L>
hipError_t launch_l(int storage, const void* fin, void* fout, const void* force, int force_mode, const GridArgs& g,
                    double omega, dim3 grid, hipStream_t s) {
  switch (storage) {
    case kF32: return launch_ls<L, kF32>(fin, fout, force, force_mode, g, omega, grid, s);
    case kF32S: return launch_ls<L, kF32S>(fin, fout, force, force_mode, g, omega, grid, s);
    case kF16S: return launch_ls<L, kF16S>(fin, fout, force, force_mode, g, omega, grid, s);
    case kBF16S: return launch_ls<L, kBF16S>(fin, fout, force, force_mode, g, omega, grid, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace

bool step_lds_eligible(int storage, const GridArgs& g) {
  const bool small_word = storage == kF32 || storage == kF32S || storage == kF16S || storage == kBF16S;
  return small_word && (g.block_x == 64 || g.block_x == 128 || g.block_x == 256) && g.nx % g.block_x == 0;
}

hipError_t launch_step_lds(int lattice, int storage, const void* fin, void* fout, const void* force, int force_mode,
                           const GridArgs& g, double omega, hipStream_t s) {
  if (!step_lds_eligible(storage, g)) return hipErrorInvalidValue;
  const uint32_t rb = 256u / g.block_x;
  const uint64_t rows = (uint64_t)g.ny * g.nzl;
  const dim3 grid((unsigned)((g.nx / g.block_x) * ((rows + rb - 1) / rb)));
  switch (lattice) {
    case kD2Q9: return launch_l<kD2Q9>(storage, fin, fout, force, force_mode, g, omega, grid, s);
    case kD3Q19: return launch_l<kD3Q19>(storage, fin, fout, force, force_mode, g, omega, grid, s);
    case kD3Q27: return launch_l<kD3Q27>(storage, fin, fout, force, force_mode, g, omega, grid, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbm

// HIP kernels (gfx950) of the lattice-Boltzmann stream-and-collide step.
//
// Paper: Bedrunka et al., arXiv:2106.12929, Sec. 2.1, Eqs. 1-4 (stream, BGK collide,
// second-order equilibrium, moments); Sec. 3.2 (differentiating the solver).
//
// Population layout ("row-interleaved SoA"): the grid is a set of rows r = z*ny + y of
// nx cells; row r stores its Q direction rows one after the other, so word (i, x) of
// row r sits at (r*Q + i)*nx + x.  Within a row every direction is a contiguous run
// along x (coalesced, vectorisable), and the Q*nx words a block writes are one
// contiguous region, which keeps the number of DRAM pages a wave touches small.
//
// Launch shape: one thread per cell, 256 threads per block covering `block_x`
// consecutive cells of a row (64, 128 or 256) and 256/block_x consecutive rows.  A
// wave never straddles two rows, so the row index, the 9 source rows of the pull
// gather and all row base addresses are wave-uniform (scalar registers); only the
// three x columns x-1, x, x+1 (periodic) are per lane.  The step is HBM-bound (about
// 1.5 flop per byte for D3Q27 FP32), so there is no MFMA; each lane moves one storage
// word per access and keeps its cell's Q populations in registers (L1/L2 absorb the
// +-1-word misalignment of the shifted loads).  Staging rows through LDS with 16-byte
// accesses speeds up a bare gather-copy but slows the full step: the LDS a block needs
// caps occupancy below what the register-resident form reaches.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>
#include <type_traits>

#include "device.h"
#include "kernels.h"
#include "lattice.h"

namespace lbm {

// ---------------------------------------------------------------------------------
// Fused pull stream + BGK collide (Eqs. 1-4), one word per lane and access.  FM selects
// the per-cell field `force` (see bgk_collide).
// ---------------------------------------------------------------------------------
// Minimum waves per SIMD asked of the compiler.  The Guo-forced f16s step needs 83
// registers unconstrained (5 waves per SIMD); asked for 6 it fits 80 with no spills.
template <int S, int FM>
struct StepMinWaves {
  static constexpr int value = (FM == kGuoForce && (S == kF16S || S == kBF16S)) ? 6 : 1;
};

template <int L, int S, int FM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(StepMinWaves<S, FM>::value))) void step_kernel(const typename Storage<S>::word* __restrict__ fin,
                                                   typename Storage<S>::word* __restrict__ fout,
                                                   const typename Storage<S>::real* __restrict__ force,
                                                   GridArgs g, typename Storage<S>::real omega) {
  using LT = Lattice<L>;
  using ST = Storage<S>;
  using real = typename ST::real;
  using CO = Coef<L, real>;
  constexpr int Q = LT::Q;
  Cell c;
  if (!cell_below(g, c, g.pitch)) return;
  // Pad lanes of a padded row (nx <= x < pitch) compute the last cell of the row again
  // (in-bounds loads, finite values) and store the result into their pad word with the
  // rest of the wave, so the row's last cache line is written by one store instruction
  // instead of two partial ones.
  Cell cs = c;
  cs.x = min(c.x, g.nx - 1);
  const Sources src = sources(cs, g);
  const size_t N = g.ncells;
  const uint32_t self = cell_index(g, cs);

  // Gather (pull streaming, Eq. 1): h_i(x) = g_i(x - c_i), as deviations from w_i.
  using W = typename ST::word;
  uint32_t xb[3];
  column_bytes<W>(src, xb);
  real d[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) d[i] = ST::to_dev(load_src<LT>(fin, g, src, xb, i), CO::W(i));

  real Fx = 0, Fy = 0, Fz = 0;
  if constexpr (FM != kNoForce) {
    Fx = force[self];
    Fy = force[N + self];
    if constexpr (LT::D == 3) Fz = force[2 * N + self];
  }
  bgk_collide<L, real, FM>(d, Fx, Fy, Fz, omega);
  const uint32_t xo = c.x * (uint32_t)sizeof(W);
#pragma unroll
  for (int i = 0; i < Q; ++i)
    store_stream(at_byte(fout + dir_row<Q>(g, c.y, c.z + g.ghost, i), xo), ST::from_dev(d[i], CO::W(i)));
}

// ---------------------------------------------------------------------------------
// Two time steps per launch for the 3D lattices (Eqs. 1-4 applied twice), with the
// intermediate populations kept in LDS: each word of the state is read from HBM once
// and written once per two steps, where two launches of step_kernel move it twice.
//
// A block owns a TX x TY tile of (x, y) columns and a chunk of z planes [zb, ze), and
// marches along z.  Per plane p it computes step t+1 on the tile plus a one-cell ring
// ((TX+2) x (TY+2) columns, gathered from HBM) and puts the rounded storage words into
// LDS; step t+2 of plane p-1 then gathers its Q populations from the LDS copies of
// planes p-2, p-1 and p.  Step t+1 of the ring columns is also computed by the
// neighbouring tiles: the price of keeping the tiles independent.
//
// The waves are specialised.  NP producer waves (one ring column per lane) load,
// collide and write plane k into LDS slot k & 1 while the NC consumer waves (one output
// cell per lane) read plane k-1 from the other slot and complete step t+2; one barrier
// per plane separates the two slots' uses.  A consumer keeps the populations of the
// two planes above its current output that it has already read (9 and 18 values): a
// plane contributes the c_z = -1 directions to the output plane below it, c_z = 0 to
// its own plane and c_z = +1 to the plane above.  The producers load plane k+1 (words
// and force; up to k+2 with three register sets) while they collide plane k; the
// consumers load the force of their next output plane one plane ahead.
//
// Each collision is bgk_collide on the words the one-step kernel would have read, and
// the intermediate words are rounded to storage exactly as its stores are, so the
// result equals two launches of step_kernel bit for bit.
//
// Tiles are 32 x 8 cells for 4-byte words and 64 x 4 for 2-byte words (a direction row
// of a tile is one 128-byte line), 32 x 4 for 8-byte words.  Consecutive tiles of a
// chunk go to the same XCD (blocks are dealt to the 8 XCDs in turn), so the ring rows
// and line ends a block shares with its neighbours are mostly served by that XCD's
// L2: a launch fetches about 1.4 times the state's bytes (two single steps fetch them
// twice); the excess is ring rows read again when a neighbouring tile is at another
// plane.
// ---------------------------------------------------------------------------------
template <int L, int S>
struct Step2Shape {
  // a tile's direction row is one 128-byte line: 32 x 8 cells for 4-byte words,
  // 64 x 4 for 2-byte words.  8-byte words take 32 x 4 tiles (rows of two lines): 6
  // waves, so that at 2 waves per SIMD a lane may hold the 256 registers the FP64
  // collisions need.
  static constexpr int WB = sizeof(typename Storage<S>::word);
  static constexpr int TX = WB == 2 ? 64 : 32, TY = WB == 8 ? 4 : 256 / TX;
  static constexpr int NSX = TX + 2, NS = NSX * (TY + 2);  // ring-tile columns
  static constexpr int NP = (NS + 63) / 64;                 // producer waves
  static constexpr int NC = TX * TY / 64;                   // consumer waves
  static constexpr int NT = 64 * (NP + NC);
  static constexpr int WAVES_PER_EU = WB == 8 ? 2 : 3;
  // The producers' plane loop.  ROTATE: passes over DEPTH rotating register sets of
  // gathers (plane p + DEPTH - 1 loading while plane p is collided); otherwise the loop
  // unrolled over two planes with a separate last plane.  Measured at 256^3 (MLUPS):
  // D3Q27 FP32 42.7k -> 43.3k rotating with two sets, shifted FP16 64.1k -> 65.3k with
  // three; the unrolled loop kept D3Q19 FP32 at 58.8k (57.4k rotating) and shifted
  // FP32 at 42.2k (41.6k).  Three sets were neutral or slower for the other forms (FP32
  // D3Q27 at 384^3 -2%: the extra registers cost its second resident block).
  static constexpr bool ROTATE = L == kD3Q27 && (S == kF32 || S == kF16S);
  static constexpr int DEPTH = L == kD3Q27 && S == kF16S ? 3 : 2;
  static constexpr int LDS = 2 * Lattice<L>::Q * NS * WB;   // the two plane slots
  // Gathers and stores through buffer resources (a 32-bit lane offset and a uniform
  // offset per access instead of a 64-bit address; 256^3, against plain pointers:
  // D3Q27 FP32 +3%, FP16 and BF16 +2%, D3Q19 FP32 +2%, BF16 +1%): every form but
  // FP64 (its resources spill scalar registers: 10% slower) and two that ran slower
  // with them, shifted FP32 D3Q27 (-4%) and D3Q19 FP16 (-2%); the kernel also leaves
  // out the velocity-shift force on 16-bit words (-1.7%).
  static constexpr bool BUFFER = WB != 8 && !(L == kD3Q27 && S == kF32S) && !(L == kD3Q19 && S == kF16S);
  // Blocks per CU the launch allows (0: as many as registers and LDS allow).  The FP32
  // D3Q27 form, whose registers allow two, runs faster at one when its tiles fit the
  // CUs (the launch decides).
  static constexpr int CAP = L == kD3Q27 && S == kF32 ? 1 : 0;
};

template <int L, int S, int FM>
__global__ __launch_bounds__((Step2Shape<L, S>::NT))
__attribute__((amdgpu_waves_per_eu(Step2Shape<L, S>::WAVES_PER_EU))) void step2_kernel(
    const typename Storage<S>::word* __restrict__ fin, typename Storage<S>::word* __restrict__ fout,
    const typename Storage<S>::real* __restrict__ force, GridArgs g, Step2Args a, typename Storage<S>::real omega) {
  using LT = Lattice<L>;
  using ST = Storage<S>;
  using W = typename ST::word;
  using real = typename ST::real;
  using CO = Coef<L, real>;
  using SH = Step2Shape<L, S>;
  constexpr int Q = LT::Q;
  constexpr int TX = SH::TX, NSX = SH::NSX, NS = SH::NS, NP = SH::NP;
  constexpr bool BUF = SH::BUFFER && !(FM == kShiftForce && SH::WB == 2);
  __shared__ W slot[2][Q][NS];

  // XCD-aware block order: blocks b, b + 8, b + 16, ... run on one XCD and take
  // consecutive tiles (a bijection of [0, nb) for any nb).
  const uint32_t nb = gridDim.x, b = blockIdx.x;
  const uint32_t per = nb / 8, extra = nb % 8, xcd = b % 8, pos = b / 8;
  const uint32_t lin = xcd < extra ? xcd * (per + 1) + pos : extra * (per + 1) + (xcd - extra) * per + pos;
  const uint32_t tx = lin % a.tiles_x, ty = (lin / a.tiles_x) % a.tiles_y, zc = lin / (a.tiles_x * a.tiles_y);
  const uint32_t x0 = tx * TX, y0 = ty * SH::TY;
  // the launch's planes [z0, z0 + nzl) in chunks of lz (all of them on a periodic grid)
  const uint32_t zb = g.z0 + zc * a.lz;
  const uint32_t ze = min(zb + a.lz, g.z0 + g.nzl);
  const uint32_t nplanes = ze - zb + 2;  // step t+1 on planes zb-1 .. ze
  const uint32_t t = threadIdx.x;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(t / 64);
  const char* fb = reinterpret_cast<const char*>(fin);
  char* ob = reinterpret_cast<char*>(fout);
  const uint32_t plane_cells = g.nx * g.ny;
  // Buffer plane of plane z (z = zb-2 .. ze+1) and force plane of plane z (zb-1 .. ze):
  // a periodic grid wraps (nz >= 3); a slab with two ghost planes on each side
  // (g.ghost == 2) keeps plane z at buffer plane z + 2 and its force at z + 1.
  const bool slab = g.ghost != 0;
  auto plane_of = [&](int z) -> uint32_t {
    if (slab) return (uint32_t)(z + 2);
    return (uint32_t)(z < 0 ? z + (int)g.nz : (z >= (int)g.nz ? z - (int)g.nz : z));
  };
  auto load_force = [&](int z, uint32_t col, real& Fx, real& Fy, real& Fz) {
    if constexpr (FM != kNoForce) {
      const uint32_t fz = slab ? (uint32_t)(z + 1) : plane_of(z);
      const real* f = force + (uint64_t)fz * plane_cells + col;
      Fx = f[0];
      Fy = f[a.force_stride];
      Fz = f[2 * a.force_stride];
    }
  };

  if (wave < (uint32_t)NP) {
    // Producer lane: ring column s (clamped lanes past the ring compute column NS - 1
    // again and write nothing).
    const bool live = t < (uint32_t)NS;
    const uint32_t s = min(t, (uint32_t)NS - 1);
    int xi = (int)x0 - 1 + (int)(s % NSX);
    int yi = (int)y0 - 1 + (int)(s / NSX);
    xi += xi < 0 ? (int)g.nx : (xi >= (int)g.nx ? -(int)g.nx : 0);
    yi += yi < 0 ? (int)g.ny : (yi >= (int)g.ny ? -(int)g.ny : 0);
    const uint32_t x = xi, y = yi, col = y * g.nx + x;
    // byte offsets inside a plane of the three source columns and rows (index c + 1
    // holds x - c, y - c)
    const uint32_t xb[3] = {wrap_inc(x, g.nx) * (uint32_t)sizeof(W), x * (uint32_t)sizeof(W),
                            wrap_dec(x, g.nx) * (uint32_t)sizeof(W)};
    const uint32_t yb[3] = {wrap_inc(y, g.ny) * a.yrow_bytes, y * a.yrow_bytes, wrap_dec(y, g.ny) * a.yrow_bytes};
    // the gathers of plane pz: the pulled words and the force
    auto load = [&](int pz, W (&r)[Q], real (&rf)[3]) {
      // the reads past plane ze (unused) read plane ze again: on a slab they stay in the
      // buffer, and the rotating loop reads up to two planes past ze
      if (SH::ROTATE || slab) pz = min(pz, (int)ze);
      const char* base[3] = {fb + (uint64_t)plane_of(pz + 1) * a.plane_bytes,
                             fb + (uint64_t)plane_of(pz) * a.plane_bytes,
                             fb + (uint64_t)plane_of(pz - 1) * a.plane_bytes};
      if constexpr (!BUF) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
          r[i] = *reinterpret_cast<const W*>(base[LT::cz(i) + 1] + (uint64_t)i * a.row_bytes +
                                             (yb[LT::cy(i) + 1] + xb[LT::cx(i) + 1]));
      } else {
        // the three source planes as buffer resources: a load takes the lane's 32-bit
        // offset and the direction row's uniform offset, no 64-bit address per load
        const __amdgpu_buffer_rsrc_t src[3] = {region_rsrc(base[0], a.plane_bytes), region_rsrc(base[1], a.plane_bytes),
                                               region_rsrc(base[2], a.plane_bytes)};
#pragma unroll
        for (int i = 0; i < Q; ++i)
          r[i] = region_load<W>(src[LT::cz(i) + 1], yb[LT::cy(i) + 1] + xb[LT::cx(i) + 1], (uint32_t)i * a.row_bytes);
      }
      load_force(pz, col, rf[0], rf[1], rf[2]);
    };
    auto produce = [&](W (&r)[Q], const real (&rf)[3], uint32_t sl) {
      real d[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) d[i] = ST::to_dev(r[i], CO::W(i));
      bgk_collide<L, real, FM>(d, rf[0], rf[1], rf[2], omega);
      if (live) {
#pragma unroll
        for (int i = 0; i < Q; ++i) slot[sl][i][s] = ST::from_dev(d[i], CO::W(i));
      }
    };
    if constexpr (SH::ROTATE) {
      // DEPTH register sets of gathers: plane p + DEPTH - 1 is loading while plane p is
      // collided (into slot p & 1) and the planes between are in flight.
      constexpr int D = SH::DEPTH;
      W r[D][Q];
      real f[D][3] = {};
#pragma unroll
      for (int d = 0; d + 1 < D; ++d) load((int)zb - 1 + d, r[d], f[d]);
      auto pass = [&](uint32_t k, auto qc) {  // plane zb-1+k, k = q mod D
        constexpr int q = decltype(qc)::value;
        load((int)(zb + k) + D - 2, r[(q + D - 1) % D], f[(q + D - 1) % D]);
        produce(r[q], f[q], D == 2 ? (uint32_t)q : k & 1);  // slot of the plane's parity
        __syncthreads();
      };
      for (uint32_t k = 0; k < nplanes; k += D) {
        pass(k, std::integral_constant<int, 0>());
        if (k + 1 >= nplanes) break;
        pass(k + 1, std::integral_constant<int, 1>());
        if constexpr (D == 3) {
          if (k + 2 >= nplanes) break;
          pass(k + 2, std::integral_constant<int, 2>());
        }
      }
    } else {
      W r0[Q], r1[Q];
      real f0[3] = {0, 0, 0}, f1[3] = {0, 0, 0};
      load((int)zb - 1, r0, f0);
      uint32_t k = 0;
      for (; k + 1 < nplanes; k += 2) {  // plane zb-1+k into slot 0, the next into slot 1
        load((int)(zb + k), r1, f1);
        produce(r0, f0, 0);
        __syncthreads();
        load((int)(zb + k) + 1, r0, f0);  // one plane past ze on the last pass: read, unused
        produce(r1, f1, 1);
        __syncthreads();
      }
      if (k < nplanes) {
        produce(r0, f0, 0);
        __syncthreads();
      }
    }
    __syncthreads();  // the consumers' last plane
  } else {
    // Consumer lane: output cell (x0 + ox, y0 + oy).
    const uint32_t u = t - 64u * NP;
    const uint32_t ox = u % TX, oy = u / TX;
    const uint32_t out_off = (y0 + oy) * a.yrow_bytes + (x0 + ox) * (uint32_t)sizeof(W);
    const uint32_t col = (y0 + oy) * g.nx + x0 + ox;
    const uint32_t l0 = (oy + 1) * NSX + ox + 1;  // own column in the ring tile
    real dA[Q], dB[Q], dC[Q];  // outputs q - 1, q, q + 1 of the plane q just read
#pragma unroll
    for (int i = 0; i < Q; ++i) dA[i] = dB[i] = dC[i] = 0;
    real cf[3] = {0, 0, 0};  // force of the next output plane, read a plane ahead
    auto consume = [&](int q, auto sl, auto emit) {
      constexpr int SL = decltype(sl)::value;
      constexpr bool EMIT = decltype(emit)::value;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const real v = ST::to_dev(slot[SL][i][l0 - (LT::cy(i) * NSX + LT::cx(i))], CO::W(i));
        if (LT::cz(i) < 0) dA[i] = v;
        if (LT::cz(i) == 0) dB[i] = v;
        if (LT::cz(i) > 0) dC[i] = v;
      }
      if constexpr (EMIT) {
        bgk_collide<L, real, FM>(dA, cf[0], cf[1], cf[2], omega);
        char* o = ob + (uint64_t)plane_of(q - 1) * a.plane_bytes;
        if constexpr (!BUF) {
#pragma unroll
          for (int i = 0; i < Q; ++i)
            store_stream(reinterpret_cast<W*>(o + (uint64_t)i * a.row_bytes + out_off), ST::from_dev(dA[i], CO::W(i)));
        } else {
          const auto ro = region_rsrc(o, a.plane_bytes);
#pragma unroll
          for (int i = 0; i < Q; ++i) store_stream(ro, out_off, (uint32_t)i * a.row_bytes, ST::from_dev(dA[i], CO::W(i)));
        }
        if (q < (int)ze) load_force(q, col, cf[0], cf[1], cf[2]);  // the next output plane's
      }
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        if (LT::cz(i) >= 0) dA[i] = dB[i];
        if (LT::cz(i) > 0) dB[i] = dC[i];
      }
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    load_force((int)zb, col, cf[0], cf[1], cf[2]);  // the first output plane's force
    __syncthreads();  // plane zb-1 written
    consume((int)zb - 1, I0(), std::false_type());
    __syncthreads();
    consume((int)zb, I1(), std::false_type());
    __syncthreads();
    uint32_t k = 2;  // planes read so far; plane zb-1+k completes output zb-2+k
    for (; k + 1 < nplanes; k += 2) {
      consume((int)(zb + k) - 1, I0(), std::true_type());
      __syncthreads();
      consume((int)(zb + k), I1(), std::true_type());
      __syncthreads();
    }
    if (k < nplanes) {
      consume((int)(zb + k) - 1, I0(), std::true_type());
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------------
// D2Q9 multiple-relaxation-time step (Sec. 3.1, Eq. 5) in the Dellar basis.
//
// The basis {1, c_x, c_y, c_x^2, c_x c_y, c_y^2, g, g c_x, g c_y}, g = (3c_x^2-1)(3c_y^2-1),
// spans the same moment subspaces as the w-orthogonal set
//   R = {1, c_x, c_y, 3c_x^2-1, c_x c_y, 3c_y^2-1, g, g c_x, g c_y}
// (the second-order rows differ from Dellar's only by multiples of the conserved rho),
// so Eq. 5's operator -M^{-1} S^{-1} (M f - m^eq) acting on f - f^eq (zero conserved
// part) is  f'_i = h_i - w_i sum_{k=3..8} R_k(c_i) n_k / (tau_k |R_k|^2),
// n_k = sum_i R_k(c_i) (h_i - f^eq_i),  |R_k|^2 = sum_i w_i R_k(c_i)^2 = 2, 1/9, 2, 4,
// 8/3, 8/3.  scale[k-3] = 1/(tau_k |R_k|^2) for uniform times.  GM selects where the
// ghost times tau_6..8 come from:
//   kGhostUniform  the uniform scales
//   kGhostField    a per-cell field ghost[3][N]
//   kGhostRelu,    the neural collision of Sec. 3.1: per cell, a network with inputs
//   kGhostTanh     x = (Pi_xx, Pi_xy, Pi_yy, N, J_x, J_y) of h - f^eq, i.e.
//                  (n_3/3, n_4, n_5/3, n_6, n_7, n_8), 53 hidden units
//                  a_j = act(b1_j + sum_k W1_jk x_k) and outputs t_n = sum_j W2_nj a_j,
//                  tau_{6+n} = exp(t_n) + 1/2.  ghost = the 530 parameters, W1 [53][6],
//                  b1 [53], W2 [3][53]; every lane reads the same addresses, so they
//                  come in through scalar loads.
// ---------------------------------------------------------------------------------
template <typename real>
__device__ __forceinline__ real act_tanh(real z) {
  return tanh(z);
}
// FP32: tanh z = 1 - 2/(e^{2z} + 1) with the hardware base-2 exponential of
// z * 2 log2(e) and the hardware reciprocal (each about 1 ulp; the reciprocal's
// argument is >= 1, never denormal).  Absolute error a few 1e-8 (relative error grows
// only where tanh z itself is below that), saturating cleanly to +-1 where e^{2z}
// overflows (1/inf = 0) or underflows.  An IEEE division here would cost a dozen VALU
// instructions per hidden unit, most of the network's cost in this VALU-bound kernel.
template <>
__device__ __forceinline__ float act_tanh<float>(float z) {
  constexpr float two_log2e = 2.0f * 1.44269504088896341f;  // exact: a power-of-two multiple
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(z * two_log2e) + 1.0f);
}
template <typename real>
__device__ __forceinline__ real exp_real(real z) {
  return exp(z);
}
template <>
__device__ __forceinline__ float exp_real<float>(float z) {
  return expf(z);
}

// The neural collision's ghost scales s_6 .. s_8 of one cell (Sec. 3.1): the network
// on x = (n_3/3, n_4, n_5/3, n_6, n_7, n_8), tau_{6+n} = exp(t_n) + 1/2,
// s = 1/(tau |R|^2).  params: the 530 parameters (W1 [53][6], b1 [53], W2 [3][53]).
template <typename real, bool RELU>
__device__ __forceinline__ void neural_scales(const MrtNoneq<real>& nq, const real* __restrict__ params, real& s6,
                                              real& s7, real& s8) {
#pragma clang fp contract(on)
  const real x[6] = {nq.nxx * real(1.0 / 3.0), nq.nxy, nq.nyy * real(1.0 / 3.0), nq.nN, nq.nJx, nq.nJy};
  const real* __restrict__ W1 = params;
  const real* __restrict__ b1 = params + kNeuralHidden * 6;
  const real* __restrict__ W2 = b1 + kNeuralHidden;
  real t0 = 0, t1 = 0, t2 = 0;
#pragma unroll
  for (int j = 0; j < kNeuralHidden; ++j) {
    real z = b1[j];
#pragma unroll
    for (int k = 0; k < 6; ++k) z += W1[6 * j + k] * x[k];
    const real act = RELU ? (z > real(0) ? z : real(0)) : act_tanh<real>(z);
    t0 += W2[j] * act;
    t1 += W2[kNeuralHidden + j] * act;
    t2 += W2[2 * kNeuralHidden + j] * act;
  }
  s6 = real(1) / (real(4) * (exp_real<real>(t0) + real(0.5)));
  s7 = real(3) / (real(8) * (exp_real<real>(t1) + real(0.5)));
  s8 = real(3) / (real(8) * (exp_real<real>(t2) + real(0.5)));
}

// ---------------------------------------------------------------------------------
// NST time steps per launch for D2Q9 (NST = 2 or 4): the 2D form of step2_kernel, with
// a pipeline of NST stages.  A block owns a segment of TX cells of x and a chunk of
// rows [yb, ye), and marches along y.  Stage s (s = 1..NST) advances the state by its
// s-th step on the segment widened by NST - s cells on each side: stage 1 gathers from
// HBM, stages 2..NST gather from the LDS ring the stage before wrote, the last stage
// writes the result.  Each stage is a group of waves, one column per lane, and runs a
// row behind the stage before: in iteration k it reads the row that stage completed in
// iteration k - 1 (a row gives the c_y = -1 directions to the row below it, c_y = 0 to
// itself, c_y = +1 to the row above; a lane keeps 3 + 6 values it has already read),
// completes the row below it and writes it to its own ring (slot k & 1).  One barrier
// per iteration.  Stage 1 loads the next row (words and force) while it collides the
// current one; the other stages read the force of their next row a row ahead.  The
// intermediate words are rounded to storage as step_kernel stores them and each
// collision is bgk_collide, so the result equals NST launches of step_kernel bit for
// bit.  The widened segments recompute 2 (NST - s) cells per row and stage: 1.008x of
// the work for NST = 2, TX = 256 and 1.023x for NST = 4, TX = 128.
// ---------------------------------------------------------------------------------
template <int TX, int NST>
struct StepNShape2D {
  static constexpr int width(int s) { return TX + 2 * (NST - s); }  // columns of stage s
  static constexpr int waves(int s) { return (width(s) + 63) / 64; }
  static constexpr int first_wave(int s) { return s == 1 ? 0 : first_wave(s - 1) + waves(s - 1); }
  static constexpr int ring(int s) { return s == 1 ? 0 : ring(s - 1) + 2 * 9 * width(s - 1); }  // words
  static constexpr int NT = 64 * first_wave(NST + 1);
  static constexpr int LDS_WORDS = ring(NST);  // rings of stages 1 .. NST-1
};

template <int S, int FM, int TX, int NST>
__global__ __launch_bounds__((StepNShape2D<TX, NST>::NT)) void stepn_2d_kernel(
    const typename Storage<S>::word* __restrict__ fin, typename Storage<S>::word* __restrict__ fout,
    const typename Storage<S>::real* __restrict__ force, GridArgs g, Step2Args a, typename Storage<S>::real omega,
    MrtScales<typename Storage<S>::real> mrt) {
  using LT = Lattice<kD2Q9>;
  using ST = Storage<S>;
  using W = typename ST::word;
  using real = typename ST::real;
  using CO = Coef<kD2Q9, real>;
  using SH = StepNShape2D<TX, NST>;
  constexpr int Q = LT::Q;
  __shared__ W lds[SH::LDS_WORDS];

  // XCD-aware block order, as in step2_kernel: consecutive segments on one XCD
  const uint32_t nb = gridDim.x, b = blockIdx.x;
  const uint32_t per = nb / 8, extra = nb % 8, xcd = b % 8, pos = b / 8;
  const uint32_t lin = xcd < extra ? xcd * (per + 1) + pos : extra * (per + 1) + (xcd - extra) * per + pos;
  const uint32_t tx = lin % a.tiles_x, yc = lin / a.tiles_x;
  const uint32_t x0 = tx * TX;
  const uint32_t yb = yc * a.lz;
  const uint32_t ye = min(yb + a.lz, g.ny);
  const uint32_t iters = (ye - yb) + 3 * (NST - 1);
  const int r0 = (int)yb - (NST - 1);  // stage 1 produces row r0 + k in iteration k
  const uint32_t t = threadIdx.x;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(t / 64);
  const char* fb = reinterpret_cast<const char*>(fin);
  char* ob = reinterpret_cast<char*>(fout);
  // rows yb-NST .. ye+NST wrapped (ny > NST)
  auto wrapy = [&](int y) -> uint32_t {
    return (uint32_t)(y < 0 ? y + (int)g.ny : (y >= (int)g.ny ? y - (int)g.ny : y));
  };
  auto wrapx = [&](int x) -> uint32_t {
    return (uint32_t)(x < 0 ? x + (int)g.nx : (x >= (int)g.nx ? x - (int)g.nx : x));
  };
  // the per-cell field a collision reads: the force (Fx, Fy) or, for kMrtField, the
  // three ghost relaxation times (tau_6, tau_7, tau_8)
  auto load_force = [&](uint32_t y, uint32_t x, real (&F)[3]) {
    if constexpr (FM == kGuoForce || FM == kShiftForce || FM == kMrtField) {
      const real* f = force + (uint64_t)y * g.nx + x;
      F[0] = f[0];
      F[1] = f[g.ncells];
      if constexpr (FM == kMrtField) F[2] = f[2 * (uint64_t)g.ncells];
    }
  };
  // the collision of one cell: BGK (forced as FM says) or the MRT collision with
  // uniform relaxation times (kMrtUniform) or per-cell ghost times (kMrtField, the
  // scales as the one-step MRT kernel forms them)
  auto collide = [&](real (&d)[Q], const real (&F)[3]) {
    if constexpr (FM == kMrtUniform) {
      mrt_relax(d, mrt_noneq(d), mrt.s);
    } else if constexpr (FM == kMrtField) {
      const MrtNoneq<real> nq = mrt_noneq(d);
      const real s[6] = {mrt.s[0], mrt.s[1], mrt.s[2], real(1) / (real(4) * F[0]), real(3) / (real(8) * F[1]),
                         real(3) / (real(8) * F[2])};
      mrt_relax(d, nq, s);
    } else {
      bgk_collide<kD2Q9, real, FM>(d, F[0], F[1], real(0), omega);
    }
  };
  // word of direction i, column j of the ring of stage s, slot sl
  auto ring_at = [&](int s, int sl, int i, int j) -> W& {
    return lds[SH::ring(s) + (sl * Q + i) * SH::width(s) + j];
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;

  if (wave < (uint32_t)SH::waves(1)) {
    // Stage 1: column s1 of the widest segment, from HBM.
    constexpr int WID = SH::width(1);
    const bool live = t < (uint32_t)WID;
    const uint32_t j = min(t, (uint32_t)WID - 1);
    const uint32_t x = wrapx((int)x0 - (NST - 1) + (int)j);
    const uint32_t xb[3] = {wrap_inc(x, g.nx) * (uint32_t)sizeof(W), x * (uint32_t)sizeof(W),
                            wrap_dec(x, g.nx) * (uint32_t)sizeof(W)};
    const uint32_t rows = (ye - yb) + 2 * (NST - 1);
    // the gathers of row py: the pulled words and the force
    auto load = [&](int py, W (&r)[Q], real (&rf)[3]) {
      py = min(py, r0 + (int)rows - 1);  // the loads past the last row read that row again
      const __amdgpu_buffer_rsrc_t src[3] = {region_rsrc(fb + (uint64_t)wrapy(py + 1) * a.yrow_bytes, a.yrow_bytes),
                                             region_rsrc(fb + (uint64_t)wrapy(py) * a.yrow_bytes, a.yrow_bytes),
                                             region_rsrc(fb + (uint64_t)wrapy(py - 1) * a.yrow_bytes, a.yrow_bytes)};
#pragma unroll
      for (int i = 0; i < Q; ++i) r[i] = region_load<W>(src[LT::cy(i) + 1], xb[LT::cx(i) + 1], (uint32_t)i * a.row_bytes);
      load_force(wrapy(py), x, rf);
    };
    auto produce = [&](uint32_t k, W (&r)[Q], const real (&rf)[3], auto sl) {
      constexpr int SL = decltype(sl)::value;
      if (k < rows) {
        real d[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = ST::to_dev(r[i], CO::W(i));
        collide(d, rf);
        if (live) {
#pragma unroll
          for (int i = 0; i < Q; ++i) ring_at(1, SL, i, j) = ST::from_dev(d[i], CO::W(i));
        }
      }
    };
    W ra[Q], rb[Q];
    real fa[3] = {0, 0, 0}, fb2[3] = {0, 0, 0};
    load(r0, ra, fa);
    uint32_t k = 0;
    for (; k + 1 < iters; k += 2) {
      load(r0 + (int)k + 1, rb, fb2);
      produce(k, ra, fa, I0());
      __syncthreads();
      load(r0 + (int)k + 2, ra, fa);
      produce(k + 1, rb, fb2, I1());
      __syncthreads();
    }
    if (k < iters) {
      produce(k, ra, fa, I0());
      __syncthreads();
    }
  } else {
    // Stages 2 .. NST: find this wave's stage (wave-uniform).
    auto run_stage = [&](auto stage) {
      constexpr int ST_ = decltype(stage)::value;
      constexpr int WID = SH::width(ST_), PWID = SH::width(ST_ - 1);
      constexpr bool LAST = ST_ == NST;
      const uint32_t lane = t - 64u * SH::first_wave(ST_);
      const bool live = lane < (uint32_t)WID;
      const uint32_t j = min(lane, (uint32_t)WID - 1);
      const uint32_t x = wrapx((int)x0 - (NST - ST_) + (int)j);
      const uint32_t out_off = x * (uint32_t)sizeof(W);
      // reads rows completed by stage ST_-1 in iterations [3 (ST_-2), ...), i.e. from
      // iteration k0 = 3 (ST_-2) + 1, and completes a row from iteration k0 + 2
      constexpr uint32_t k0 = 3 * (ST_ - 2) + 1;
      const uint32_t rows = (ye - yb) + 2 * (NST - ST_);
      real dA[Q], dB[Q], dC[Q];  // rows q - 1, q, q + 1 of the row q just read
#pragma unroll
      for (int i = 0; i < Q; ++i) dA[i] = dB[i] = dC[i] = 0;
      // force of the next row this stage completes, read a row ahead
      real cf[3] = {0, 0, 0};
      load_force(wrapy(r0 + (int)(k0 + 2) - 2 * (ST_ - 1)), x, cf);
      auto step = [&](uint32_t k, auto sl) {
        constexpr int SL = decltype(sl)::value;  // slot written in iteration k (k & 1)
        if (k < k0 || k >= k0 + 2 + rows) return;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const real v = ST::to_dev(ring_at(ST_ - 1, 1 - SL, i, (int)j + 1 - LT::cx(i)), CO::W(i));
          if (LT::cy(i) < 0) dA[i] = v;
          if (LT::cy(i) == 0) dB[i] = v;
          if (LT::cy(i) > 0) dC[i] = v;
        }
        if (k >= k0 + 2) {
          // the row completed here: stage ST_ produces row r0 + k - 2 (ST_ - 1)
          const int row = r0 + (int)k - 2 * (ST_ - 1);
          collide(dA, cf);
          if (k + 1 < k0 + 2 + rows) load_force(wrapy(row + 1), x, cf);
          if constexpr (LAST) {
            if (live) {
              const auto o = region_rsrc(ob + (uint64_t)row * a.yrow_bytes, a.yrow_bytes);
#pragma unroll
              for (int i = 0; i < Q; ++i)
                store_stream(o, out_off, (uint32_t)i * a.row_bytes, ST::from_dev(dA[i], CO::W(i)));
            }
          } else if (live) {
#pragma unroll
            for (int i = 0; i < Q; ++i) ring_at(ST_, SL, i, j) = ST::from_dev(dA[i], CO::W(i));
          }
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          if (LT::cy(i) >= 0) dA[i] = dB[i];
          if (LT::cy(i) > 0) dB[i] = dC[i];
        }
      };
      uint32_t k = 0;
      for (; k + 1 < iters; k += 2) {
        step(k, I0());
        __syncthreads();
        step(k + 1, I1());
        __syncthreads();
      }
      if (k < iters) {
        step(k, I0());
        __syncthreads();
      }
      (void)PWID;
    };
    if constexpr (NST == 2) {
      run_stage(std::integral_constant<int, 2>());
    } else {
      static_assert(NST == 4, "2 or 4 stages");
      if (wave < (uint32_t)SH::first_wave(3))
        run_stage(std::integral_constant<int, 2>());
      else if (wave < (uint32_t)SH::first_wave(4))
        run_stage(std::integral_constant<int, 3>());
      else
        run_stage(std::integral_constant<int, 4>());
    }
  }
}

// One D2Q9 MRT step (the collision and GM as described above the D2Q9 multi-step kernel).
template <int S, int GM>
__global__ __launch_bounds__(256) void mrt_step_kernel(const typename Storage<S>::word* __restrict__ fin,
                                                       typename Storage<S>::word* __restrict__ fout,
                                                       const typename Storage<S>::real* __restrict__ ghost,
                                                       GridArgs g, MrtScales<typename Storage<S>::real> sc) {
  using LT = Lattice<kD2Q9>;
  using ST = Storage<S>;
  using real = typename ST::real;
  using CO = Coef<kD2Q9, real>;
  constexpr int Q = 9;
  Cell c;
  if (!cell_of_thread(g, c)) return;
  const Sources src = sources(c, g);
  const size_t N = g.ncells;
  uint32_t xb[3];
  column_bytes<typename ST::word>(src, xb);

  real d[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) d[i] = ST::to_dev(load_src<LT>(fin, g, src, xb, i), CO::W(i));
  const MrtNoneq<real> nq = mrt_noneq(d);
  real s6 = real(sc.s[3]), s7 = real(sc.s[4]), s8 = real(sc.s[5]);
  if constexpr (GM == kGhostField) {
    const uint32_t n = cell_index(g, c);
    s6 = real(1) / (real(4) * ghost[n]);
    s7 = real(3) / (real(8) * ghost[N + n]);
    s8 = real(3) / (real(8) * ghost[2 * N + n]);
  } else if constexpr (GM == kGhostRelu || GM == kGhostTanh) {
    neural_scales<real, GM == kGhostRelu>(nq, ghost, s6, s7, s8);
  }
  const real s[6] = {sc.s[0], sc.s[1], sc.s[2], s6, s7, s8};
  mrt_relax(d, nq, s);
  const uint32_t xo = c.x * (uint32_t)sizeof(typename ST::word);
#pragma unroll
  for (int i = 0; i < Q; ++i) store_stream(at_byte(fout + dir_row<Q>(g, c.y, c.z, i), xo), ST::from_dev(d[i], CO::W(i)));
}

// ---------------------------------------------------------------------------------
// Streaming only: raw word permutation (bit-exact for every storage kind).
// ---------------------------------------------------------------------------------
template <int L, typename W>
__global__ __launch_bounds__(256) void stream_kernel(const W* __restrict__ fin, W* __restrict__ fout, GridArgs g) {
  using LT = Lattice<L>;
  Cell c;
  if (!cell_of_thread(g, c)) return;
  const Sources src = sources(c, g);
#pragma unroll
  for (int i = 0; i < LT::Q; ++i) store_stream(&fout[dir_row<LT::Q>(g, c.y, c.z, i) + c.x], fin[src_offset<LT>(g, src, i)]);
}

// The transpose of streaming, on real words: out_i(x) = in_i(x + c_i).
template <int L, typename W>
__global__ __launch_bounds__(256) void unstream_kernel(const W* __restrict__ fin, W* __restrict__ fout, GridArgs g) {
  using LT = Lattice<L>;
  Cell c;
  if (!cell_of_thread(g, c)) return;
  const Sources src = sources(c, g);
#pragma unroll
  for (int i = 0; i < LT::Q; ++i) store_stream(&fout[dir_row<LT::Q>(g, c.y, c.z, i) + c.x], fin[rev_offset<LT>(g, src, i)]);
}

// ---------------------------------------------------------------------------------
// Equilibrium initialisation (Eq. 3) in FP64, one rounding to storage.
// ---------------------------------------------------------------------------------
template <int L, int S>
__global__ __launch_bounds__(256) void init_kernel(const double* __restrict__ rho_in, const double* __restrict__ u,
                                                   typename Storage<S>::word* __restrict__ fout, GridArgs g) {
  using LT = Lattice<L>;
  using ST = Storage<S>;
  Cell c;
  if (!cell_of_thread(g, c)) return;
  const size_t N = g.ncells;
  const uint32_t n = cell_index(g, c);
  const double rho = rho_in ? rho_in[n] : 1.0;
  const double ux = u[n], uy = u[N + n], uz = LT::D == 3 ? u[2 * N + n] : 0.0;
  const double usq = 1.5 * (ux * ux + uy * uy + uz * uz);
#pragma unroll
  for (int i = 0; i < LT::Q; ++i) {
    const double cu = LT::cx(i) * ux + LT::cy(i) * uy + LT::cz(i) * uz;
    const double dev = LT::w(i) * ((rho - 1.0) + rho * (3.0 * cu + 4.5 * cu * cu - usq));
    // unshifted storage keeps f = W_i + dev with the base the kernels subtract again
    store_stream(&fout[dir_row<LT::Q>(g, c.y, c.z, i) + c.x],
                 ST::from_f64_dev(dev, static_cast<double>(Coef<L, typename ST::real>::W(i))));
  }
}

// ---------------------------------------------------------------------------------
// Moments (Eq. 4) and FP64 reductions, one thread per cell (the launch of the step
// kernels).  The reductions fold in a fixed order that depends on the grid only, so every
// call sums the same way: a DPP reduction per wave (wave_fold, total in lane 63), the
// block's four waves in order, then blocks in consecutive runs of kFoldBlock
// (fold_partials_kernel), then those run results (reduce_partials_kernel).
// ---------------------------------------------------------------------------------
template <typename real>
struct CellMoments {
  real drho, rho, u[3];
};

// Moments of one cell from its Q stored words and its force F (zero when unforced).
template <int L, int S>
__device__ __forceinline__ CellMoments<typename Storage<S>::real> moments_of_words(
    const typename Storage<S>::word (&w)[Lattice<L>::Q], const typename Storage<S>::real (&F)[3]) {
  using LT = Lattice<L>;
  using ST = Storage<S>;
  using real = typename ST::real;
  real drho = 0, j[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < LT::Q; ++i) {
    const real d = ST::to_dev(w[i], Coef<L, real>::W(i));
    drho += d;
    add_times(j[0], LT::cx(i), d);
    add_times(j[1], LT::cy(i), d);
    add_times(j[2], LT::cz(i), d);
  }
#pragma unroll
  for (int a = 0; a < LT::D; ++a) j[a] -= real(0.5) * F[a];
  CellMoments<real> m;
  m.drho = drho;
  m.rho = real(1) + drho;
  const real inv = real(1) / m.rho;
#pragma unroll
  for (int a = 0; a < 3; ++a) m.u[a] = j[a] * inv;
  return m;
}

// The Q words of the cell at column x of a row whose direction rows start at `row`
// (word (i, x) at row[i*pitch + x]), and, if FORCED, its force (cell index n of the
// [D][N] field); F = 0 otherwise.
template <int L, int S, bool FORCED>
__device__ __forceinline__ void load_cell(const typename Storage<S>::word* __restrict__ row,
                                          const typename Storage<S>::real* __restrict__ force, size_t N,
                                          uint32_t pitch, uint32_t x, uint32_t n,
                                          typename Storage<S>::word (&w)[Lattice<L>::Q],
                                          typename Storage<S>::real (&F)[3]) {
  using W = typename Storage<S>::word;
  const uint32_t xo = x * (uint32_t)sizeof(W);
#pragma unroll
  for (int i = 0; i < Lattice<L>::Q; ++i) w[i] = *at_byte(row + (uint64_t)i * pitch, xo);
#pragma unroll
  for (int a = 0; a < 3; ++a) F[a] = 0;
  if constexpr (FORCED) {
#pragma unroll
    for (int a = 0; a < Lattice<L>::D; ++a) F[a] = force[a * N + n];
  }
}

template <int L, int S>
__device__ __forceinline__ CellMoments<typename Storage<S>::real> cell_moments(
    const typename Storage<S>::word* __restrict__ row, const typename Storage<S>::real* __restrict__ force,
    size_t N, uint32_t pitch, uint32_t x, uint32_t n) {
  typename Storage<S>::word w[Lattice<L>::Q];
  typename Storage<S>::real F[3];
  if (force)
    load_cell<L, S, true>(row, force, N, pitch, x, n, w, F);
  else
    load_cell<L, S, false>(row, force, N, pitch, x, n, w, F);
  return moments_of_words<L, S>(w, F);
}

// Reduction operator of entry k of the kNred results: max for max|u|, min for min rho,
// sum otherwise.
__device__ __forceinline__ double red_op(int k, double a, double b) {
  return k == 6 ? fmax(a, b) : k == 7 ? fmin(a, b) : a + b;
}

// The value of entry k that leaves the other operand of red_op unchanged.
__device__ __forceinline__ double red_idle(int k) { return k == 7 ? 1.0e300 : 0.0; }

// A DPP move of a double (its two 32-bit halves moved alike); lanes of rows outside
// ROWS keep `idle`.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_move(double v, double idle) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v), o = __builtin_bit_cast(uint64_t, idle);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)b, CTRL, ROWS, 0xF, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(b >> 32), CTRL, ROWS, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Folds entry k over the 64 lanes of a full wave; lane 63 ends with the wave's result.
// Lane pairs (quad_perm 1,0,3,2), then quad pairs (quad_perm 2,3,0,1), then quads of a
// 16-lane row (row_ror 4 and 8) leave each row's result in all its lanes; row_bcast15
// adds row 0 into row 1 and row 2 into row 3, row_bcast31 adds row 1 into row 3.  These
// are register moves between lanes, so the fold takes no LDS bandwidth.
__device__ __forceinline__ double wave_fold(int k, double v) {
  const double idle = red_idle(k);
  v = red_op(k, v, dpp_move<0xB1, 0xF>(v, idle));
  v = red_op(k, v, dpp_move<0x4E, 0xF>(v, idle));
  v = red_op(k, v, dpp_move<0x124, 0xF>(v, idle));
  v = red_op(k, v, dpp_move<0x128, 0xF>(v, idle));
  v = red_op(k, v, dpp_move<0x142, 0xA>(v, idle));
  v = red_op(k, v, dpp_move<0x143, 0xC>(v, idle));
  return v;
}

template <int L, int S, bool FORCED, bool REDUCE, uint32_t SPAN>
__global__ __launch_bounds__(256) void moments_kernel(const typename Storage<S>::word* __restrict__ f,
                                                      const typename Storage<S>::real* __restrict__ force,
                                                      typename Storage<S>::real* __restrict__ rho_out,
                                                      typename Storage<S>::real* __restrict__ u_out,
                                                      double* __restrict__ partials, GridArgs g) {
  using LT = Lattice<L>;
  using W = typename Storage<S>::word;
  using R = typename Storage<S>::real;
  constexpr int Q = LT::Q;
  const size_t N = g.ncells;
  // acc: [0] sum drho, [1..3] sum rho u, [4] 1/2 sum |u|^2, [5] non-finite, [6] max|u|^2 (the
  // block's partial takes its square root once: sqrt is monotonic and correctly rounded, so
  // that is max|u| exactly), [7] min rho
  double acc[kNred] = {0, 0, 0, 0, 0, 0, 0, 1.0e300};
  // A block walks SPAN consecutive blocks of cells, each thread summing its cells in
  // order, so that the fold below is paid once per SPAN cells of a thread.
#pragma unroll 1
  for (uint32_t j = 0; j < SPAN; ++j) {
    Cell c;
    // no early return: every thread joins the block's fold
    if (!cell_in_block(g, c, g.nx, blockIdx.x * SPAN + j)) continue;
    const uint32_t r = c.z * g.ny + c.y;
    W w[Q];
    R F[3];
    load_cell<L, S, FORCED>(f + (uint64_t)r * Q * g.pitch, force, N, g.pitch, c.x, r * g.nx + c.x, w, F);
    const auto m = moments_of_words<L, S>(w, F);
    const uint32_t xo = c.x * (uint32_t)sizeof(R);  // row-uniform base + lane byte offset
    if (rho_out) store_stream(at_byte(rho_out + (uint64_t)r * g.nx, xo), m.rho);
    if (u_out) {
#pragma unroll
      for (int k = 0; k < LT::D; ++k) store_stream(at_byte(u_out + k * N + (uint64_t)r * g.nx, xo), m.u[k]);
    }
    if constexpr (REDUCE) {
      const double rho = m.rho;
      const double ux = m.u[0], uy = m.u[1], uz = m.u[2];
      const double usq = ux * ux + uy * uy + uz * uz;
      if (isfinite(rho) && isfinite(usq)) {
        acc[0] += (double)m.drho;
        acc[1] += rho * ux;
        acc[2] += rho * uy;
        acc[3] += rho * uz;
        acc[4] += 0.5 * usq;
        acc[6] = fmax(acc[6], usq);
        acc[7] = fmin(acc[7], rho);
      } else {
        acc[5] += 1.0;
      }
    }
  }
  if constexpr (REDUCE) {
#pragma unroll
    for (int k = 0; k < kNred; ++k) acc[k] = wave_fold(k, acc[k]);
    __shared__ double sh[4][kNred];
    if (threadIdx.x % 64 == 63) {
#pragma unroll
      for (int k = 0; k < kNred; ++k) sh[threadIdx.x / 64][k] = acc[k];
    }
    __syncthreads();
    if (threadIdx.x < kNred) {
      const int k = threadIdx.x;
      double v = sh[0][k];
      for (int wv = 1; wv < 4; ++wv) v = red_op(k, v, sh[wv][k]);
      partials[(uint64_t)blockIdx.x * kNred + k] = k == 6 ? sqrt(v) : v;
    }
  }
}

// Second stage: block j folds partials [j kFoldBlock, (j + 1) kFoldBlock) into out[j]:
// thread t takes 8 consecutive entries in order, then a fixed tree over the threads.
__global__ __launch_bounds__(256) void fold_partials_kernel(const double* __restrict__ in, uint64_t n_in,
                                                            double* __restrict__ out) {
  double acc[kNred] = {0, 0, 0, 0, 0, 0, 0, 1.0e300};
  const uint64_t base = (uint64_t)blockIdx.x * kFoldBlock + threadIdx.x * 8u;
  for (int m = 0; m < 8; ++m) {
    if (base + m < n_in) {
#pragma unroll
      for (int k = 0; k < kNred; ++k) acc[k] = red_op(k, acc[k], in[(base + m) * kNred + k]);
    }
  }
  __shared__ double sh[kNred][256];
#pragma unroll
  for (int k = 0; k < kNred; ++k) sh[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int k = 0; k < kNred; ++k) sh[k][threadIdx.x] = red_op(k, sh[k][threadIdx.x], sh[k][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x < kNred) out[(uint64_t)blockIdx.x * kNred + threadIdx.x] = sh[threadIdx.x][0];
}

// One block folds the per-block partials in a fixed order; adds N to turn sum(drho)
// into the mass.
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double* __restrict__ partials, int nblocks,
                                                              double* __restrict__ red, double ncells) {
  __shared__ double sh[kNred][256];
  double acc[kNred] = {0, 0, 0, 0, 0, 0, 0, 1.0e300};
  for (int b = threadIdx.x; b < nblocks; b += 256) {
#pragma unroll
    for (int k = 0; k < kNred; ++k) {
      const double v = partials[b * kNred + k];
      acc[k] = k == 6 ? fmax(acc[k], v) : k == 7 ? fmin(acc[k], v) : acc[k] + v;
    }
  }
#pragma unroll
  for (int k = 0; k < kNred; ++k) sh[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int k = 0; k < kNred; ++k) {
        const double a = sh[k][threadIdx.x], b = sh[k][threadIdx.x + s];
        sh[k][threadIdx.x] = k == 6 ? fmax(a, b) : k == 7 ? fmin(a, b) : a + b;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    red[0] = ncells + sh[0][0];
    for (int k = 1; k < kNred; ++k) red[k] = sh[k][0];
  }
}

// ---------------------------------------------------------------------------------
// Adjoint of one step.  The forward collision, with h = S g_t gathered, rho = 1 + drho,
// u = (sum c h + F/2)/rho and deq_i = W_i drho + rho (A_i c_i.u + B_i (c_i.u)^2 -
// W_i 3/2 |u|^2), is g'_i = (1 - omega) h_i + omega deq_i + G_i with the Guo source
// G_i = (1 - omega/2)(A_i c_i.F - 3 W_i u.F + 2 B_i (c_i.u)(c_i.F)).  With lam' =
// lam_next(x) and the weighted moments
//   mW = sum W_i lam'_i,  mA_a = sum A_i c_ia lam'_i,  mB_ab = sum B_i c_ia c_ib lam'_i
// its transpose is
//   P   = omega (mW + u.mA + u.mB.u - 3/2 |u|^2 mW)                    (via drho)
//   V_a = omega rho (mA_a + 2 (mB u)_a - 3 u_a mW)
//         + (1 - omega/2)(2 (mB F)_a - 3 F_a mW)                        (via u)
//   mu_j = (1 - omega) lam'_j + P + sum_a V_a (c_ja - u_a) / rho
//   dF_a = (1 - omega/2)(mA_a - 3 u_a mW + 2 (mB u)_a) + V_a / (2 rho)
// and lam_t,j(x - c_j) = mu_j(x): the transpose of the pull gather is a scatter to the
// same addresses, each written exactly once (no atomics).
//
// MODE selects where lam' comes from and where mu goes:
//   kAdjScatter:    lam' = lam_next(x) (aligned);  lam_t,j(x - c_j) = mu_j (scattered)
//   kAdjLocalLam:   lam' = lam_next(x) (aligned);  chi_t(x) = mu (aligned)
//   kAdjLocalChi:   lam'_i = chi_next_i(x + c_i)  (gathered: lam_{t+1} = S^T chi_{t+1});
//                   chi_t(x) = mu (aligned)
// In the local ("chi") form every store is aligned; lam_t = S^T chi_t.
// ---------------------------------------------------------------------------------
// J_C(h)^T of one cell's BGK collision (with Guo force when FORCED), applied in place:
// d holds the pulled populations h_i - w_i, lam the adjoint lambda_{t+1} at the cell on
// entry and mu = J_C(h)^T lambda_{t+1} on exit; (ax, ay, az) returns (dg'/dF)^T lambda,
// the cell's force-gradient contribution.  The Jacobian depends on h through rho and u
// only, so the work splits into adjoint_moments (of d) and adjoint_apply (on lam).
// Products are fused only within an expression, so every kernel that inlines them
// rounds identically.
template <typename real>
struct AdjMoments {
  real rho, inv_rho, ux, uy, uz;
};

template <int L, typename real, bool FORCED>
__device__ __forceinline__ AdjMoments<real> adjoint_moments(const real (&d)[Lattice<L>::Q], real Fx, real Fy,
                                                            real Fz) {
#pragma clang fp contract(on)
  using LT = Lattice<L>;
  constexpr int Q = LT::Q;
  real drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    drho += d[i];
    add_times(jx, LT::cx(i), d[i]);
    add_times(jy, LT::cy(i), d[i]);
    add_times(jz, LT::cz(i), d[i]);
  }
  if constexpr (FORCED) {
    jx += real(0.5) * Fx;
    jy += real(0.5) * Fy;
    jz += real(0.5) * Fz;
  }
  AdjMoments<real> m;
  m.rho = real(1) + drho;
  m.inv_rho = real(1) / m.rho;
  m.ux = jx * m.inv_rho;
  m.uy = jy * m.inv_rho;
  m.uz = jz * m.inv_rho;
  return m;
}

template <int L, typename real, bool FORCED>
__device__ __forceinline__ void adjoint_apply(const AdjMoments<real>& m, real (&lam)[Lattice<L>::Q], real Fx, real Fy,
                                              real Fz, real omega, real& ax, real& ay, real& az) {
#pragma clang fp contract(on)
  using LT = Lattice<L>;
  using CO = Coef<L, real>;
  constexpr int Q = LT::Q;
  const real rho = m.rho, inv_rho = m.inv_rho, ux = m.ux, uy = m.uy, uz = m.uz;
  real mW = 0, mAx = 0, mAy = 0, mAz = 0, bxx = 0, byy = 0, bzz = 0, bxy = 0, bxz = 0, byz = 0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const real l = lam[i];
    const int cx = LT::cx(i), cy = LT::cy(i), cz = LT::cz(i);
    const real al = CO::A(i) * l, bl = CO::B(i) * l;
    mW += CO::W(i) * l;
    add_times(mAx, cx, al);
    add_times(mAy, cy, al);
    add_times(mAz, cz, al);
    add_times(bxx, cx * cx, bl);
    add_times(byy, cy * cy, bl);
    add_times(bzz, cz * cz, bl);
    add_times(bxy, cx * cy, bl);
    add_times(bxz, cx * cz, bl);
    add_times(byz, cy * cz, bl);
  }
  const real mBux = bxx * ux + bxy * uy + bxz * uz;
  const real mBuy = bxy * ux + byy * uy + byz * uz;
  const real mBuz = bxz * ux + byz * uy + bzz * uz;
  const real usq15 = real(1.5) * (ux * ux + uy * uy + uz * uz);
  const real P = omega * (mW + ux * mAx + uy * mAy + uz * mAz + ux * mBux + uy * mBuy + uz * mBuz - usq15 * mW);
  const real orho = omega * rho;
  real Vx = orho * (mAx + real(2) * mBux - real(3) * ux * mW);
  real Vy = orho * (mAy + real(2) * mBuy - real(3) * uy * mW);
  real Vz = orho * (mAz + real(2) * mBuz - real(3) * uz * mW);
  const real guo = real(1) - real(0.5) * omega;
  if constexpr (FORCED) {
    const real mBFx = bxx * Fx + bxy * Fy + bxz * Fz;
    const real mBFy = bxy * Fx + byy * Fy + byz * Fz;
    const real mBFz = bxz * Fx + byz * Fy + bzz * Fz;
    Vx += guo * (real(2) * mBFx - real(3) * Fx * mW);
    Vy += guo * (real(2) * mBFy - real(3) * Fy * mW);
    Vz += guo * (real(2) * mBFz - real(3) * Fz * mW);
  }
  const real vx = Vx * inv_rho, vy = Vy * inv_rho, vz = Vz * inv_rho;
  const real base = P - (vx * ux + vy * uy + vz * uz);
  const real keep = real(1) - omega;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    real mu = keep * lam[j] + base;
    if (LT::cx(j) > 0) mu += vx;
    if (LT::cx(j) < 0) mu -= vx;
    if (LT::cy(j) > 0) mu += vy;
    if (LT::cy(j) < 0) mu -= vy;
    if (LT::cz(j) > 0) mu += vz;
    if (LT::cz(j) < 0) mu -= vz;
    lam[j] = mu;
  }
  if constexpr (FORCED) {
    const real half_inv = real(0.5) * inv_rho;
    ax = guo * (mAx - real(3) * ux * mW + real(2) * mBux) + Vx * half_inv;
    ay = guo * (mAy - real(3) * uy * mW + real(2) * mBuy) + Vy * half_inv;
    az = guo * (mAz - real(3) * uz * mW + real(2) * mBuz) + Vz * half_inv;
  } else {
    ax = ay = az = 0;
  }
}

template <int L, typename real, bool FORCED>
__device__ __forceinline__ void adjoint_collide(const real (&d)[Lattice<L>::Q], real (&lam)[Lattice<L>::Q], real Fx,
                                                real Fy, real Fz, real omega, real& ax, real& ay, real& az) {
  adjoint_apply<L, real, FORCED>(adjoint_moments<L, real, FORCED>(d, Fx, Fy, Fz), lam, Fx, Fy, Fz, omega, ax, ay, az);
}

template <int L, int S, bool FORCED, int MODE>
__global__ __launch_bounds__(256) void adjoint_kernel(const typename Storage<S>::word* __restrict__ gt,
                                                      const typename Storage<S>::real* __restrict__ lam_next,
                                                      typename Storage<S>::real* __restrict__ lam_out,
                                                      const typename Storage<S>::real* __restrict__ force,
                                                      typename Storage<S>::real* __restrict__ dforce, GridArgs g,
                                                      typename Storage<S>::real omega) {
  using LT = Lattice<L>;
  using ST = Storage<S>;
  using real = typename ST::real;
  using CO = Coef<L, real>;
  constexpr int Q = LT::Q;
  Cell c;
  if (!cell_of_thread(g, c)) return;
  const Sources src = sources(c, g);
  const size_t N = g.ncells;
  const uint32_t self = cell_index(g, c);

  uint32_t xw[3], xr[3];  // column byte offsets for storage words and for reals
  column_bytes<typename ST::word>(src, xw);
  column_bytes<real>(src, xr);
  real d[Q], lam[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) d[i] = ST::to_dev(load_src<LT>(gt, g, src, xw, i), CO::W(i));
#pragma unroll
  for (int i = 0; i < Q; ++i)
    lam[i] = MODE == kAdjLocalChi ? load_rev<LT>(lam_next, g, src, xr, i)
                                  : *at_byte(lam_next + dir_row<Q>(g, c.y, c.z, i), xr[1]);
  real Fx = 0, Fy = 0, Fz = 0;
  if constexpr (FORCED) {
    Fx = force[self];
    Fy = force[N + self];
    if constexpr (LT::D == 3) Fz = force[2 * N + self];
  }
  real ax, ay, az;
  adjoint_collide<L, real, FORCED>(d, lam, Fx, Fy, Fz, omega, ax, ay, az);
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    if constexpr (MODE == kAdjScatter) {
      // shifted rows: a wave's store straddles cache lines that the neighbouring wave
      // completes, so it stays a plain (cached) store for the halves to merge in L2
      *at_byte(lam_out + dir_row<Q>(g, src.y[LT::cy(j) + 1], src.z[LT::cz(j) + 1], j), xr[LT::cx(j) + 1]) = lam[j];
    } else {
      store_stream(at_byte(lam_out + dir_row<Q>(g, c.y, c.z, j), xr[1]), lam[j]);
    }
  }
  if constexpr (FORCED) {
    if (dforce) {
      dforce[self] += ax;
      dforce[N + self] += ay;
      if constexpr (LT::D == 3) dforce[2 * N + self] += az;
    }
  }
}

// ---------------------------------------------------------------------------------
// Two adjoint steps per launch (collision-local form, chi in and chi out):
//   chi_t   = J_C(S g_t)^T   S^T chi_{t+1}   (on a tile plus a one-cell ring, into LDS)
//   chi_t-1 = J_C(S g_t-1)^T S^T chi_t       (on the tile, from LDS, to HBM)
// with the force gradient of both steps added in the order of two one-step launches,
// (dF + a_t) + a_t-1.  The structure is step2_kernel's (tiles of 32 x 8 columns marching
// along z, producer and consumer waves, two LDS slots, one barrier per plane), with the
// adjoint's transposed streaming: lambda_i(x) = chi_i(x + c_i), so a plane of chi_t
// gives its c_z = +1 directions to the output plane below it.  Producers gather the
// state g_t (pull), chi_t+1 (transposed) and the force from HBM, one plane ahead;
// consumers gather g_t-1, the force and the force gradient from HBM (also one plane
// ahead) and chi_t from LDS.  The producers also leave a_t of the tile's own cells in
// LDS for the consumers.  Each cell's arithmetic is that of adjoint_collide, as in
// adjoint_kernel, so the result equals two of its launches bit for bit.
// ---------------------------------------------------------------------------------
template <int L, int S, bool FORCED>
__global__ __launch_bounds__((Step2Shape<L, kF32>::NT)) __attribute__((amdgpu_waves_per_eu(3))) void adjoint2_kernel(
    const typename Storage<S>::word* __restrict__ gt, const typename Storage<S>::word* __restrict__ gtm1,
    const typename Storage<S>::real* __restrict__ chi_next, typename Storage<S>::real* __restrict__ chi_out,
    const typename Storage<S>::real* __restrict__ force, typename Storage<S>::real* __restrict__ dforce, GridArgs g,
    Step2Args aw, Step2Args ar, typename Storage<S>::real omega) {
  using LT = Lattice<L>;
  using ST = Storage<S>;
  using W = typename ST::word;
  using real = typename ST::real;
  using CO = Coef<L, real>;
  using SH = Step2Shape<L, kF32>;  // tiles by the 4-byte adjoint reals
  constexpr int Q = LT::Q;
  constexpr int TX = SH::TX, TY = SH::TY, NSX = SH::NSX, NS = SH::NS, NP = SH::NP;
  __shared__ real slot[2][Q][NS];
  __shared__ real stash[2][3][TX * TY];  // a_t of the tile's cells, by plane

  const uint32_t nb = gridDim.x, b = blockIdx.x;
  const uint32_t per = nb / 8, extra = nb % 8, xcd = b % 8, pos = b / 8;
  const uint32_t lin = xcd < extra ? xcd * (per + 1) + pos : extra * (per + 1) + (xcd - extra) * per + pos;
  const uint32_t tx = lin % ar.tiles_x, ty = (lin / ar.tiles_x) % ar.tiles_y, zc = lin / (ar.tiles_x * ar.tiles_y);
  const uint32_t x0 = tx * TX, y0 = ty * TY;
  const uint32_t zb = zc * ar.lz;
  const uint32_t ze = min(zb + ar.lz, g.nz);
  const uint32_t nplanes = ze - zb + 2;  // chi_t on planes zb-1 .. ze
  const uint32_t t = threadIdx.x;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(t / 64);
  const char* fbt = reinterpret_cast<const char*>(gt);
  const char* fbm = reinterpret_cast<const char*>(gtm1);
  const char* cbn = reinterpret_cast<const char*>(chi_next);
  char* cbo = reinterpret_cast<char*>(chi_out);
  const uint32_t plane_cells = g.nx * g.ny;
  const bool grad = FORCED && dforce != nullptr;
  auto wrapz = [&](int z) -> uint32_t {
    return (uint32_t)(z < 0 ? z + (int)g.nz : (z >= (int)g.nz ? z - (int)g.nz : z));
  };
  auto load_force = [&](uint32_t z, uint32_t col, real& Fx, real& Fy, real& Fz) {
    if constexpr (FORCED) {
      const real* f = force + (uint64_t)z * plane_cells + col;
      Fx = f[0];
      Fy = f[g.ncells];
      Fz = f[2 * g.ncells];
    }
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;

  if (wave < (uint32_t)NP) {
    // Producer lane: ring column s.
    const bool live = t < (uint32_t)NS;
    const uint32_t s = min(t, (uint32_t)NS - 1);
    const uint32_t sx = s % NSX, sy = s / NSX;
    int xi = (int)x0 - 1 + (int)sx;
    int yi = (int)y0 - 1 + (int)sy;
    xi += xi < 0 ? (int)g.nx : (xi >= (int)g.nx ? -(int)g.nx : 0);
    yi += yi < 0 ? (int)g.ny : (yi >= (int)g.ny ? -(int)g.ny : 0);
    const uint32_t x = xi, y = yi, col = y * g.nx + x;
    // own cell of the tile (its a_t is kept for the consumers)
    const bool own = live && sx >= 1 && sx <= (uint32_t)TX && sy >= 1 && sy <= (uint32_t)TY;
    const uint32_t own_idx = (sy - 1) * TX + (sx - 1);
    // index c + 1: pull sources x - c (words), transposed sources x + c (reals)
    const uint32_t xw[3] = {wrap_inc(x, g.nx) * (uint32_t)sizeof(W), x * (uint32_t)sizeof(W),
                            wrap_dec(x, g.nx) * (uint32_t)sizeof(W)};
    const uint32_t yw[3] = {wrap_inc(y, g.ny) * aw.yrow_bytes, y * aw.yrow_bytes, wrap_dec(y, g.ny) * aw.yrow_bytes};
    const uint32_t xr[3] = {wrap_dec(x, g.nx) * (uint32_t)sizeof(real), x * (uint32_t)sizeof(real),
                            wrap_inc(x, g.nx) * (uint32_t)sizeof(real)};
    const uint32_t yr[3] = {wrap_dec(y, g.ny) * ar.yrow_bytes, y * ar.yrow_bytes, wrap_inc(y, g.ny) * ar.yrow_bytes};
    // the gathers of plane pz: state words pulled from g_t, chi_t+1 transposed, force
    auto load = [&](int pz, W (&rw)[Q], real (&rc)[Q], real (&rf)[3]) {
      const char* base[3] = {fbt + (uint64_t)wrapz(pz + 1) * aw.plane_bytes, fbt + (uint64_t)wrapz(pz) * aw.plane_bytes,
                             fbt + (uint64_t)wrapz(pz - 1) * aw.plane_bytes};
#pragma unroll
      for (int i = 0; i < Q; ++i)
        rw[i] = *reinterpret_cast<const W*>(base[LT::cz(i) + 1] + (uint64_t)i * aw.row_bytes +
                                            (yw[LT::cy(i) + 1] + xw[LT::cx(i) + 1]));
      const char* cb[3] = {cbn + (uint64_t)wrapz(pz - 1) * ar.plane_bytes, cbn + (uint64_t)wrapz(pz) * ar.plane_bytes,
                           cbn + (uint64_t)wrapz(pz + 1) * ar.plane_bytes};
#pragma unroll
      for (int i = 0; i < Q; ++i)
        rc[i] = *reinterpret_cast<const real*>(cb[LT::cz(i) + 1] + (uint64_t)i * ar.row_bytes +
                                               (yr[LT::cy(i) + 1] + xr[LT::cx(i) + 1]));
      load_force(wrapz(pz), col, rf[0], rf[1], rf[2]);
    };
    auto moments = [&](const W (&rw)[Q], const real (&rf)[3]) {
      real d[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) d[i] = ST::to_dev(rw[i], CO::W(i));
      return adjoint_moments<L, real, FORCED>(d, rf[0], rf[1], rf[2]);
    };
    auto finish = [&](const AdjMoments<real>& m, real (&lam)[Q], const real (&rf)[3], auto sl) {
      constexpr int SL = decltype(sl)::value;
      real ax, ay, az;
      adjoint_apply<L, real, FORCED>(m, lam, rf[0], rf[1], rf[2], omega, ax, ay, az);
      if (live) {
#pragma unroll
        for (int i = 0; i < Q; ++i) slot[SL][i][s] = lam[i];
      }
      if (grad && own) {
        stash[SL][0][own_idx] = ax;
        stash[SL][1][own_idx] = ay;
        stash[SL][2][own_idx] = az;
      }
    };
    // A plane's state words are reduced to rho and u before the next plane's gathers
    // are issued (fewer registers held); those gathers are then in flight while the
    // plane's adjoint is applied and the barrier waited on.
    W w0[Q], w1[Q];
    real c0[Q], c1[Q];
    real f0[3] = {0, 0, 0}, f1[3] = {0, 0, 0};
    load((int)zb - 1, w0, c0, f0);
    uint32_t k = 0;
    for (; k + 1 < nplanes; k += 2) {
      const AdjMoments<real> m0 = moments(w0, f0);
      load((int)(zb + k), w1, c1, f1);
      finish(m0, c0, f0, I0());
      __syncthreads();
      const AdjMoments<real> m1 = moments(w1, f1);
      load((int)(zb + k) + 1, w0, c0, f0);  // one plane past ze on the last pass: read, unused
      finish(m1, c1, f1, I1());
      __syncthreads();
    }
    if (k < nplanes) {
      const AdjMoments<real> m0 = moments(w0, f0);
      finish(m0, c0, f0, I0());
      __syncthreads();
    }
    __syncthreads();  // the consumers' last plane
  } else {
    // Consumer lane: output cell (x0 + ox, y0 + oy).
    const uint32_t u = t - 64u * NP;
    const uint32_t ox = u % TX, oy = u / TX;
    const uint32_t x = x0 + ox, y = y0 + oy, col = y * g.nx + x;
    const uint32_t out_off = y * ar.yrow_bytes + x * (uint32_t)sizeof(real);
    const uint32_t l0 = (oy + 1) * NSX + ox + 1;
    const uint32_t xw[3] = {wrap_inc(x, g.nx) * (uint32_t)sizeof(W), x * (uint32_t)sizeof(W),
                            wrap_dec(x, g.nx) * (uint32_t)sizeof(W)};
    const uint32_t yw[3] = {wrap_inc(y, g.ny) * aw.yrow_bytes, y * aw.yrow_bytes, wrap_dec(y, g.ny) * aw.yrow_bytes};
    real dA[Q], dB[Q], dC[Q];  // lambda of outputs q - 1, q, q + 1 for the chi_t plane q just read
#pragma unroll
    for (int i = 0; i < Q; ++i) dA[i] = dB[i] = dC[i] = 0;
    // the next output plane's gathers, issued a plane ahead: g_t-1 pulled (raw words),
    // its force and the force gradient it adds to
    W st[Q];
    real sf[3] = {0, 0, 0}, sg[3] = {0, 0, 0};
    auto load_next = [&](int oz) {
      const char* base[3] = {fbm + (uint64_t)wrapz(oz + 1) * aw.plane_bytes, fbm + (uint64_t)wrapz(oz) * aw.plane_bytes,
                             fbm + (uint64_t)wrapz(oz - 1) * aw.plane_bytes};
#pragma unroll
      for (int i = 0; i < Q; ++i)
        st[i] = *reinterpret_cast<const W*>(base[LT::cz(i) + 1] + (uint64_t)i * aw.row_bytes +
                                            (yw[LT::cy(i) + 1] + xw[LT::cx(i) + 1]));
      load_force((uint32_t)oz, col, sf[0], sf[1], sf[2]);
      if (grad) {
        const real* f = dforce + (uint64_t)oz * plane_cells + col;
        sg[0] = f[0];
        sg[1] = f[g.ncells];
        sg[2] = f[2 * g.ncells];
      }
    };
    real atx = 0, aty = 0, atz = 0;  // a_t of the next output plane
    real ntx = 0, nty = 0, ntz = 0;
    auto consume = [&](int qz, auto sl, auto emit) {
      constexpr int SL = decltype(sl)::value;
      constexpr bool EMIT = decltype(emit)::value;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const real v = slot[SL][i][l0 + (LT::cy(i) * NSX + LT::cx(i))];
        if (LT::cz(i) > 0) dA[i] = v;
        if (LT::cz(i) == 0) dB[i] = v;
        if (LT::cz(i) < 0) dC[i] = v;
      }
      if (grad) {
        ntx = stash[SL][0][u];
        nty = stash[SL][1][u];
        ntz = stash[SL][2][u];
      }
      if constexpr (EMIT) {
        const int oz = qz - 1;  // the output plane completed by plane qz
        real d[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) d[i] = ST::to_dev(st[i], CO::W(i));
        real ax, ay, az;
        adjoint_collide<L, real, FORCED>(d, dA, sf[0], sf[1], sf[2], omega, ax, ay, az);
        char* o = cbo + (uint64_t)oz * ar.plane_bytes + out_off;
#pragma unroll
        for (int i = 0; i < Q; ++i) store_stream(reinterpret_cast<real*>(o + (uint64_t)i * ar.row_bytes), dA[i]);
        if (grad) {
          real* f = dforce + (uint64_t)oz * plane_cells + col;
          f[0] = (sg[0] + atx) + ax;
          f[g.ncells] = (sg[1] + aty) + ay;
          f[2 * g.ncells] = (sg[2] + atz) + az;
        }
        if (oz + 1 < (int)ze) load_next(oz + 1);
      }
      atx = ntx;
      aty = nty;
      atz = ntz;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        if (LT::cz(i) <= 0) dA[i] = dB[i];
        if (LT::cz(i) < 0) dB[i] = dC[i];
      }
    };
    load_next((int)zb);  // the first output plane
    __syncthreads();  // plane zb-1 written
    consume((int)zb - 1, I0(), std::false_type());
    __syncthreads();
    consume((int)zb, I1(), std::false_type());
    __syncthreads();
    uint32_t k = 2;  // planes read so far; plane zb-1+k completes output zb-2+k
    for (; k + 1 < nplanes; k += 2) {
      consume((int)(zb + k) - 1, I0(), std::true_type());
      __syncthreads();
      consume((int)(zb + k), I1(), std::true_type());
      __syncthreads();
    }
    if (k < nplanes) {
      consume((int)(zb + k) - 1, I0(), std::true_type());
      __syncthreads();
    }
  }
}

// Adjoint of the moments map (rho, u) = (sum g, (sum c g - F/2)/rho).
template <int L, int S>
__global__ __launch_bounds__(256) void moments_adjoint_kernel(const typename Storage<S>::word* __restrict__ f,
                                                              const typename Storage<S>::real* __restrict__ force,
                                                              const typename Storage<S>::real* __restrict__ drho_in,
                                                              const typename Storage<S>::real* __restrict__ du_in,
                                                              typename Storage<S>::real* __restrict__ lam_out,
                                                              typename Storage<S>::real* __restrict__ dforce,
                                                              GridArgs g) {
  using LT = Lattice<L>;
  using real = typename Storage<S>::real;
  Cell c;
  if (!cell_of_thread(g, c)) return;
  const size_t N = g.ncells;
  const uint32_t n = cell_index(g, c);
  const uint64_t row = dir_row<LT::Q>(g, c.y, c.z, 0);
  const auto m = cell_moments<L, S>(f + row, force, N, g.pitch, c.x, n);
  const real inv = real(1) / m.rho;
  const real dr = drho_in ? drho_in[n] : real(0);
  real du[3] = {0, 0, 0};
  if (du_in) {
#pragma unroll
    for (int a = 0; a < LT::D; ++a) du[a] = du_in[a * N + n];
  }
  const real bx = du[0] * inv, by = du[1] * inv, bz = du[2] * inv;
  const real base = dr - (bx * m.u[0] + by * m.u[1] + bz * m.u[2]);
#pragma unroll
  for (int j = 0; j < LT::Q; ++j) {
    real v = base;
    if (LT::cx(j) > 0) v += bx;
    if (LT::cx(j) < 0) v -= bx;
    if (LT::cy(j) > 0) v += by;
    if (LT::cy(j) < 0) v -= by;
    if (LT::cz(j) > 0) v += bz;
    if (LT::cz(j) < 0) v -= bz;
    store_stream(&lam_out[row + (uint64_t)j * g.pitch + c.x], v);
  }
  if (dforce) {
#pragma unroll
    for (int a = 0; a < LT::D; ++a) dforce[a * N + n] -= real(0.5) * du[a] * inv;
  }
}

// ---------------------------------------------------------------------------------
// Host-side launchers (template dispatch over lattice x storage x forced).
// ---------------------------------------------------------------------------------
static dim3 cell_grid(const GridArgs& g) {
  const uint32_t blocks_x = (g.nx + g.block_x - 1) / g.block_x;
  const uint64_t rows = (uint64_t)g.ny * g.nzl;
  const uint32_t rows_per_block = 256u / g.block_x;
  return dim3((unsigned)(blocks_x * ((rows + rows_per_block - 1) / rows_per_block)));
}

// ---------------------------------------------------------------------------------
// Resident-block caps.  Several kernels move more bytes per second with fewer blocks
// resident on a CU than their register use would allow (FP64 steps 69% -> 74% of
// 8 TB/s at two blocks instead of five, the forced collision-local adjoints 70-72% ->
// 73-76% at three): how fast HBM serves a kernel depends on how many rows are read and
// written at once, not only on how many loads are in flight.  The cap is a dynamic LDS
// reservation that the kernels never touch: with 160 KB of LDS per CU, a block that
// reserves 64, 48, 36, 30 or 24 KB leaves room for at most 2, 3, 4, 5 or 6 blocks.
// Each table entry is the cap that measured fastest for that instantiation at its
// benchmark size (256^3 for the 3D lattices, 8192^2 for D2Q9; caps 1-6 against none,
// then the chosen cap against none again on a near-equilibrium state, three passes; the
// figures quoted are those of the second measurement).  0 keeps the register-limited
// occupancy, which won or tied everywhere else: the FP32 D3Q27 step, the 16-bit steps,
// whose gain on zero-filled buffers (up to 4%) did not hold on a real state, and the
// D2Q9 FP32 step, whose 1% gain on a random state turned into a 5% loss on the
// benchmark's Taylor-Green state.
// ---------------------------------------------------------------------------------
constexpr size_t kLdsPerCu = 160 * 1024;
constexpr size_t reserve_for_cap(int cap) {
  return cap == 2 ? 64 * 1024 : cap == 3 ? 48 * 1024 : cap == 4 ? 36 * 1024 : cap == 5 ? 30 * 1024
       : cap == 6 ? 24 * 1024 : 0;
}
static_assert(2 * reserve_for_cap(2) <= kLdsPerCu && 3 * reserve_for_cap(2) > kLdsPerCu, "cap 2");
static_assert(3 * (reserve_for_cap(3) + 256) <= kLdsPerCu && 4 * reserve_for_cap(3) > kLdsPerCu, "cap 3");
static_assert(4 * reserve_for_cap(4) <= kLdsPerCu && 5 * reserve_for_cap(4) > kLdsPerCu, "cap 4");
static_assert(5 * reserve_for_cap(5) <= kLdsPerCu && 6 * reserve_for_cap(5) > kLdsPerCu, "cap 5");
static_assert(6 * reserve_for_cap(6) <= kLdsPerCu && 7 * reserve_for_cap(6) > kLdsPerCu, "cap 6");

template <int L, int S, int FM>
constexpr int step_cap() {
  if (S == kF64) return L == kD2Q9 ? 3 : 2;  // D3Q27 68.5 -> 73.4%, forced 70 -> 74.7%, D3Q19 70.2 -> 75.0%, D2Q9 72.6 -> 77.8%
  if (L == kD3Q27 && FM == kGuoForce && S == kF32S) return 2;  // 72.4 -> 75.3%
  return 0;
}

template <int L, int S, bool FORCED, int MODE>
constexpr int adjoint_cap() {
  if (L != kD3Q27) return 0;
  if (MODE == kAdjScatter) return (S == kF32 || S == kF16S) ? 2 : 0;  // 65.4 -> 67.4%, 66.5 -> 70.1%
  if (MODE == kAdjLocalLam) return 0;
  if (S == kF64) return 2;  // 70.9 -> 73.8%, forced 68.1 -> 73.9%
  return FORCED ? 3 : 0;    // forced f32 69.8 -> 72.8%, f16s 71.8 -> 75.5%, bf16s 71.8 -> 74.0%
}

template <int S, int GM>
constexpr int mrt_cap() {
  return (S == kF64 && GM == kGhostUniform) ? 3 : 0;  // 73.0 -> 77.7%
}

template <int L, int S, bool FORCED, bool REDUCE, uint32_t SPAN>
constexpr int moments_cap() {
  if (L != kD3Q27 || FORCED || SPAN != 1) return 0;
  if (REDUCE) return S == kF32 ? 3 : 0;                         // 69.1 -> 74.2%
  return S == kF32 ? 2 : S == kF16S ? 4 : S == kF64 ? 2 : 0;  // 70.2 -> 76.8%, 72.7 -> 77.6%, 72.0 -> 74.4%
}

template <int L, int S>
static hipError_t launch_step_ls(const void* fin, void* fout, const void* force, int force_mode, const GridArgs& g,
                                 double omega, hipStream_t s) {
  using ST = Storage<S>;
  using W = typename ST::word;
  using R = typename ST::real;
  const dim3 grid = cell_grid(g);
  if (!force || force_mode == kNoForce)
    step_kernel<L, S, kNoForce><<<grid, 256, reserve_for_cap(step_cap<L, S, kNoForce>()), s>>>(
        (const W*)fin, (W*)fout, nullptr, g, (R)omega);
  else if (force_mode == kGuoForce)
    step_kernel<L, S, kGuoForce><<<grid, 256, reserve_for_cap(step_cap<L, S, kGuoForce>()), s>>>(
        (const W*)fin, (W*)fout, (const R*)force, g, (R)omega);
  else if (force_mode == kShiftForce)
    step_kernel<L, S, kShiftForce><<<grid, 256, reserve_for_cap(step_cap<L, S, kShiftForce>()), s>>>(
        (const W*)fin, (W*)fout, (const R*)force, g, (R)omega);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Multi-step launches for every storage kind: on the 3D lattices step2_kernel (one
// launch at 256^3 against two of step_kernel: FP32 and shifted FP32 1.47-1.59x, shifted
// FP16 and BF16 1.10-1.30x, FP64 1.5x), on D2Q9 stepn_2d_kernel.
template <int L, int S>
constexpr bool step2_enabled() {
  if (L == kD2Q9) return true;
  return L == kD3Q27 || L == kD3Q19;
}

// Segment width of the D2Q9 multi-step kernel advancing nst steps (0: none fits).
static uint32_t stepn_2d_width(const GridArgs& g, int nst) {
  if (g.ny < (uint32_t)nst + 1) return 0;  // rows wrap once at most
  if (nst == 4) return g.nx % 128 == 0 ? 128 : g.nx % 64 == 0 ? 64 : 0;
  return g.nx % 256 == 0 ? 256 : g.nx % 64 == 0 ? 64 : 0;
}

template <int L, int S>
static bool step2_fits(const GridArgs& g) {
  if constexpr (!step2_enabled<L, S>()) {
    return false;
  } else if constexpr (L == kD2Q9) {
    // the Q direction rows of a grid row are one region with 32-bit offsets
    const uint64_t yrow = (uint64_t)Lattice<L>::Q * g.pitch * sizeof(typename Storage<S>::word);
    return g.ghost == 0 && g.z0 == 0 && g.nzl == g.nz && stepn_2d_width(g, 2) != 0 && yrow < (uint64_t(1) << 32);
  } else {
    using SH = Step2Shape<L, S>;
    const uint64_t plane = (uint64_t)g.ny * Lattice<L>::Q * g.pitch * sizeof(typename Storage<S>::word);
    return g.ghost == 0 && g.z0 == 0 && g.nzl == g.nz && g.nx % SH::TX == 0 && g.ny % SH::TY == 0 && g.nz >= 3 &&
           plane < (uint64_t(1) << 32);
  }
}

// Compute units of the current device (cached per device).
static uint32_t device_cus() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int n = cache[dev].load(std::memory_order_relaxed);
  if (n <= 0) {
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cache[dev].store(n, std::memory_order_relaxed);
  }
  return (uint32_t)n;
}

// Planes (rows in 2D) per chunk: the length that minimises rounds * (lz + extra), the
// duration of the launch if each block takes lz + extra plane-times (its chunk plus the
// planes its pipeline fills and drains: 2 for the 3D two-step kernel, 3 (NST - 1) for
// the 2D NST-step kernel) and `slots` blocks run at once.
static uint32_t step2_chunk(uint64_t tiles, uint32_t nz, uint64_t slots, uint32_t extra) {
  uint32_t best = nz;
  uint64_t best_cost = ~uint64_t(0);
  for (uint32_t lz = 8;; lz += 8) {
    const uint32_t l = lz < nz ? lz : nz;
    const uint64_t blocks = tiles * ((nz + l - 1) / l);
    const uint64_t cost = ((blocks + slots - 1) / slots) * (l + extra);
    if (cost < best_cost) {
      best_cost = cost;
      best = l;
    }
    if (l == nz) break;
  }
  return best;
}

// Blocks of one multi-step instantiation resident per CU (its registers and LDS decide;
// the D3Q27 forms take one block of 10 or 11 waves per CU at 99-168 registers, 6 waves
// at up to 256 for FP64, the D3Q19 forms up to two).
template <typename K>
static uint32_t blocks_per_cu(std::atomic<int>& cached, K kernel, int threads, size_t dyn_lds = 0) {
  int n = cached.load(std::memory_order_relaxed);
  if (n <= 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, dyn_lds) != hipSuccess || n <= 0) n = 1;
    cached.store(n, std::memory_order_relaxed);
  }
  return (uint32_t)n;
}

// The dynamic LDS a two-step launch reserves (untouched) to hold it to its block cap.
template <int L, int S>
constexpr size_t step2_reserve() {
  using SH = Step2Shape<L, S>;
  static_assert(SH::CAP == 0 || SH::CAP == 1, "a cap of one block");
  return SH::CAP == 1 && (size_t)SH::LDS <= kLdsPerCu / 2 ? kLdsPerCu / 2 + 1024 - SH::LDS : 0;
}

template <int L, int S, int FM>
static uint32_t step2_blocks_per_cu(bool capped) {
  static std::atomic<int> cached[2] = {{0}, {0}};
  return blocks_per_cu(cached[capped], step2_kernel<L, S, FM>, Step2Shape<L, S>::NT,
                       capped ? step2_reserve<L, S>() : 0);
}

template <int S, int FM, int TX, int NST>
static hipError_t launch_stepn_2d(const void* fin, void* fout, const void* force, const GridArgs& g, double omega,
                                  hipStream_t s, const double* mrt_scales = nullptr) {
  using ST = Storage<S>;
  using W = typename ST::word;
  using R = typename ST::real;
  static std::atomic<int> cached{0};
  MrtScales<R> sc;
  for (int k = 0; k < 6; ++k) sc.s[k] = mrt_scales ? (R)mrt_scales[k] : R(0);
  Step2Args a;
  a.tiles_x = g.nx / TX;
  a.tiles_y = 1;
  a.row_bytes = g.pitch * (uint32_t)sizeof(W);
  a.yrow_bytes = Lattice<kD2Q9>::Q * a.row_bytes;
  a.plane_bytes = 0;
  const uint64_t slots =
      (uint64_t)blocks_per_cu(cached, stepn_2d_kernel<S, FM, TX, NST>, StepNShape2D<TX, NST>::NT) * device_cus();
  a.lz = step2_chunk(a.tiles_x, g.ny, slots, 3 * (NST - 1));
  const dim3 grid((unsigned)(a.tiles_x * ((g.ny + a.lz - 1) / a.lz)));
  stepn_2d_kernel<S, FM, TX, NST><<<grid, StepNShape2D<TX, NST>::NT, 0, s>>>((const W*)fin, (W*)fout,
                                                                             (const R*)force, g, a, (R)omega, sc);
  return hipGetLastError();
}

template <int S, int FM, int NST>
static hipError_t launch_stepn_2d_w(const void* fin, void* fout, const void* force, const GridArgs& g, double omega,
                                    hipStream_t s, const double* mrt_scales = nullptr) {
  constexpr int WIDE = NST == 4 ? 128 : 256;
  if (stepn_2d_width(g, NST) == WIDE)
    return launch_stepn_2d<S, FM, WIDE, NST>(fin, fout, force, g, omega, s, mrt_scales);
  return launch_stepn_2d<S, FM, 64, NST>(fin, fout, force, g, omega, s, mrt_scales);
}

template <int S>
static hipError_t launch_stepn_mrt_s(int nst, const void* fin, void* fout, const GridArgs& g, const double* scales,
                                     const void* ghost, hipStream_t s) {
  if (!step2_fits<kD2Q9, S>(g) || (nst != 2 && nst != 4) || (nst == 4 && stepn_2d_width(g, 4) == 0))
    return hipErrorInvalidValue;
  if (ghost) {
    if (nst == 4) return launch_stepn_2d_w<S, kMrtField, 4>(fin, fout, ghost, g, 0.0, s, scales);
    return launch_stepn_2d_w<S, kMrtField, 2>(fin, fout, ghost, g, 0.0, s, scales);
  }
  if (nst == 4) return launch_stepn_2d_w<S, kMrtUniform, 4>(fin, fout, nullptr, g, 0.0, s, scales);
  return launch_stepn_2d_w<S, kMrtUniform, 2>(fin, fout, nullptr, g, 0.0, s, scales);
}

template <int L, int S, int FM>
static hipError_t launch_step2_lsf(const void* fin, void* fout, const void* force, const GridArgs& g, double omega,
                                   hipStream_t s) {
  using ST = Storage<S>;
  using W = typename ST::word;
  using R = typename ST::real;
  using SH = Step2Shape<L, S>;
  Step2Args a;
  a.tiles_x = g.nx / SH::TX;
  a.tiles_y = g.ny / SH::TY;
  a.row_bytes = g.pitch * (uint32_t)sizeof(W);
  a.yrow_bytes = Lattice<L>::Q * a.row_bytes;
  a.plane_bytes = g.ny * a.yrow_bytes;
  // a slab's force has a ghost plane below and above its own planes
  a.force_stride = g.ghost ? (uint64_t)g.nx * g.ny * (g.nz + 2) : g.ncells;
  const uint64_t tiles = (uint64_t)a.tiles_x * a.tiles_y;
  // The block cap holds where every tile then runs its whole plane range in one round
  // (FP32 D3Q27 256^3: +1.6%); with more tiles than CUs a second resident block fills
  // the rounds' tails (384^3: 3% faster uncapped; 320^3 and 512^3 alike either way).
  const bool capped = SH::CAP == 1 && tiles <= device_cus();
  a.lz = step2_chunk(tiles, g.nzl, (uint64_t)step2_blocks_per_cu<L, S, FM>(capped) * device_cus(), 2);
  const dim3 grid((unsigned)(tiles * ((g.nzl + a.lz - 1) / a.lz)));
  step2_kernel<L, S, FM><<<grid, SH::NT, capped ? step2_reserve<L, S>() : 0, s>>>((const W*)fin, (W*)fout,
                                                                                  (const R*)force, g, a, (R)omega);
  return hipGetLastError();
}

// Two steps on a z-slab with two ghost planes on each side (g.ghost == 2): the 3D
// lattices and the tiles of the periodic two-step launches, nz >= 2, the planes
// [z0, z0 + nzl) of the slab.
template <int L, int S>
static bool step2_slab_fits(const GridArgs& g) {
  if constexpr (!step2_enabled<L, S>() || L == kD2Q9) {
    return false;
  } else {
    using SH = Step2Shape<L, S>;
    const uint64_t plane = (uint64_t)g.ny * Lattice<L>::Q * g.pitch * sizeof(typename Storage<S>::word);
    return g.ghost == 2 && g.nzl >= 1 && g.z0 + g.nzl <= g.nz && g.nx % SH::TX == 0 && g.ny % SH::TY == 0 &&
           g.nz >= 2 && plane < (uint64_t(1) << 32);
  }
}

template <int L, int S>
static hipError_t step2_slab_fits_ls(const GridArgs& g, bool* ok) {
  *ok = step2_slab_fits<L, S>(g);
  return hipSuccess;
}

template <int L, int S>
static hipError_t launch_stepn_ls(int nst, const void* fin, void* fout, const void* force, int force_mode,
                                  const GridArgs& g, double omega, hipStream_t s) {
  if constexpr (!step2_enabled<L, S>()) {
    return hipErrorInvalidValue;
  } else {
    if (!step2_fits<L, S>(g) || (nst != 2 && nst != 4)) return hipErrorInvalidValue;
    if (nst == 4 && (L != kD2Q9 || stepn_2d_width(g, 4) == 0)) return hipErrorInvalidValue;
    if (force_mode != kNoForce && force_mode != kGuoForce && force_mode != kShiftForce) return hipErrorInvalidValue;
    const int fm = force ? force_mode : kNoForce;
    if constexpr (L == kD2Q9) {
      if (nst == 4) {
        if (fm == kNoForce) return launch_stepn_2d_w<S, kNoForce, 4>(fin, fout, nullptr, g, omega, s);
        if (fm == kGuoForce) return launch_stepn_2d_w<S, kGuoForce, 4>(fin, fout, force, g, omega, s);
        return launch_stepn_2d_w<S, kShiftForce, 4>(fin, fout, force, g, omega, s);
      }
      if (fm == kNoForce) return launch_stepn_2d_w<S, kNoForce, 2>(fin, fout, nullptr, g, omega, s);
      if (fm == kGuoForce) return launch_stepn_2d_w<S, kGuoForce, 2>(fin, fout, force, g, omega, s);
      return launch_stepn_2d_w<S, kShiftForce, 2>(fin, fout, force, g, omega, s);
    } else {
      if (nst != 2) return hipErrorInvalidValue;
      if (fm == kNoForce) return launch_step2_lsf<L, S, kNoForce>(fin, fout, nullptr, g, omega, s);
      if (fm == kGuoForce) return launch_step2_lsf<L, S, kGuoForce>(fin, fout, force, g, omega, s);
      return launch_step2_lsf<L, S, kShiftForce>(fin, fout, force, g, omega, s);
    }
  }
}

// Four steps per launch on D2Q9 for FP64, FP32 and shifted FP32 (8192^2: 2.8-3.2x two
// single steps' rate, against 1.7-1.8x for two steps per launch); shifted FP16 ran
// slower with four (226.6k against 243.7k MLUPS: its conversions make the deeper
// pipeline arithmetic-bound) and takes two.
template <int L, int S>
static hipError_t launch_step2_slab_ls(const void* fin, void* fout, const void* force, int force_mode,
                                       const GridArgs& g, double omega, hipStream_t s) {
  if constexpr (!step2_enabled<L, S>() || L == kD2Q9) {
    return hipErrorInvalidValue;
  } else {
    if (!step2_slab_fits<L, S>(g)) return hipErrorInvalidValue;
    if (force_mode != kNoForce && force_mode != kGuoForce && force_mode != kShiftForce) return hipErrorInvalidValue;
    const int fm = force ? force_mode : kNoForce;
    if (fm == kNoForce) return launch_step2_lsf<L, S, kNoForce>(fin, fout, nullptr, g, omega, s);
    if (fm == kGuoForce) return launch_step2_lsf<L, S, kGuoForce>(fin, fout, force, g, omega, s);
    return launch_step2_lsf<L, S, kShiftForce>(fin, fout, force, g, omega, s);
  }
}

template <int L, int S>
static hipError_t max_steps_ls(const GridArgs& g, int* n) {
  constexpr bool FOUR = L == kD2Q9;
  *n = !step2_fits<L, S>(g) ? 1 : (FOUR && stepn_2d_width(g, 4) != 0) ? 4 : 2;
  return hipSuccess;
}

template <int S>
static hipError_t launch_mrt_s(const void* fin, void* fout, const void* ghost, int ghost_mode, const GridArgs& g,
                               const double* scales, hipStream_t s) {
  using ST = Storage<S>;
  using W = typename ST::word;
  using R = typename ST::real;
  MrtScales<R> sc;
  for (int k = 0; k < 6; ++k) sc.s[k] = (R)scales[k];
  const W* a = (const W*)fin;
  W* b = (W*)fout;
  const R* gh = (const R*)ghost;
  switch (ghost_mode) {
    case kGhostUniform:
      mrt_step_kernel<S, kGhostUniform><<<cell_grid(g), 256, reserve_for_cap(mrt_cap<S, kGhostUniform>()), s>>>(
          a, b, nullptr, g, sc);
      break;
    case kGhostField: mrt_step_kernel<S, kGhostField><<<cell_grid(g), 256, 0, s>>>(a, b, gh, g, sc); break;
    case kGhostRelu: mrt_step_kernel<S, kGhostRelu><<<cell_grid(g), 256, 0, s>>>(a, b, gh, g, sc); break;
    case kGhostTanh: mrt_step_kernel<S, kGhostTanh><<<cell_grid(g), 256, 0, s>>>(a, b, gh, g, sc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_stepn_mrt(int storage, int nst, const void* fin, void* fout, const GridArgs& g,
                            const double* scales, const void* ghost, hipStream_t s) {
  switch (storage) {
    case kF64: return launch_stepn_mrt_s<kF64>(nst, fin, fout, g, scales, ghost, s);
    case kF32: return launch_stepn_mrt_s<kF32>(nst, fin, fout, g, scales, ghost, s);
    case kF32S: return launch_stepn_mrt_s<kF32S>(nst, fin, fout, g, scales, ghost, s);
    case kF16S: return launch_stepn_mrt_s<kF16S>(nst, fin, fout, g, scales, ghost, s);
    case kBF16S: return launch_stepn_mrt_s<kBF16S>(nst, fin, fout, g, scales, ghost, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_mrt(int storage, const void* fin, void* fout, const void* ghost, int ghost_mode, const GridArgs& g,
                      const double* scales, hipStream_t s) {
  switch (storage) {
    case kF64: return launch_mrt_s<kF64>(fin, fout, ghost, ghost_mode, g, scales, s);
    case kF32: return launch_mrt_s<kF32>(fin, fout, ghost, ghost_mode, g, scales, s);
    case kF32S: return launch_mrt_s<kF32S>(fin, fout, ghost, ghost_mode, g, scales, s);
    case kF16S: return launch_mrt_s<kF16S>(fin, fout, ghost, ghost_mode, g, scales, s);
    case kBF16S: return launch_mrt_s<kBF16S>(fin, fout, ghost, ghost_mode, g, scales, s);
  }
  return hipErrorInvalidValue;
}

template <int L, int S, int MODE>
static hipError_t launch_adjoint_lsm(const void* gt, const void* lam_next, void* lam_out, const void* force,
                                     void* dforce, const GridArgs& g, double omega, hipStream_t s) {
  using ST = Storage<S>;
  using W = typename ST::word;
  using R = typename ST::real;
  if (force)
    adjoint_kernel<L, S, true, MODE><<<cell_grid(g), 256, reserve_for_cap(adjoint_cap<L, S, true, MODE>()), s>>>(
        (const W*)gt, (const R*)lam_next, (R*)lam_out, (const R*)force, (R*)dforce, g, (R)omega);
  else
    adjoint_kernel<L, S, false, MODE><<<cell_grid(g), 256, reserve_for_cap(adjoint_cap<L, S, false, MODE>()), s>>>(
        (const W*)gt, (const R*)lam_next, (R*)lam_out, nullptr, nullptr, g, (R)omega);
  return hipGetLastError();
}

template <int L, int S>
static hipError_t launch_adjoint_ls(int mode, const void* gt, const void* lam_next, void* lam_out, const void* force,
                                    void* dforce, const GridArgs& g, double omega, hipStream_t s) {
  switch (mode) {
    case kAdjScatter: return launch_adjoint_lsm<L, S, kAdjScatter>(gt, lam_next, lam_out, force, dforce, g, omega, s);
    case kAdjLocalLam: return launch_adjoint_lsm<L, S, kAdjLocalLam>(gt, lam_next, lam_out, force, dforce, g, omega, s);
    case kAdjLocalChi: return launch_adjoint_lsm<L, S, kAdjLocalChi>(gt, lam_next, lam_out, force, dforce, g, omega, s);
  }
  return hipErrorInvalidValue;
}

// Two adjoint steps per launch (adjoint2_kernel): the 3D lattices, every storage kind
// of the state but FP64 (the adjoint reals are FP32 then), on the grids the two-step
// forward kernel's 32 x 8 tiles take.
template <int L, int S>
static bool adjoint2_fits(const GridArgs& g) {
  if constexpr ((L != kD3Q27 && L != kD3Q19) || S == kF64) {
    return false;
  } else {
    using SH = Step2Shape<L, kF32>;
    const uint64_t plane = (uint64_t)g.ny * Lattice<L>::Q * g.pitch * sizeof(typename Storage<S>::real);
    return g.ghost == 0 && g.z0 == 0 && g.nzl == g.nz && g.nx % SH::TX == 0 && g.ny % SH::TY == 0 && g.nz >= 3 &&
           plane < (uint64_t(1) << 32);
  }
}

template <int L, int S>
static hipError_t adjoint2_fits_ls(const GridArgs& g, bool* ok) {
  *ok = adjoint2_fits<L, S>(g);
  return hipSuccess;
}

template <int L, int S, bool FORCED>
static uint32_t adjoint2_blocks_per_cu() {
  static std::atomic<int> cached{0};
  return blocks_per_cu(cached, adjoint2_kernel<L, S, FORCED>, Step2Shape<L, kF32>::NT);
}

template <int L, int S>
static hipError_t launch_adjoint2_ls(const void* gt, const void* gtm1, const void* chi_next, void* chi_out,
                                     const void* force, void* dforce, const GridArgs& g, double omega, hipStream_t s) {
  if constexpr ((L != kD3Q27 && L != kD3Q19) || S == kF64) {
    return hipErrorInvalidValue;
  } else {
    using ST = Storage<S>;
    using W = typename ST::word;
    using R = typename ST::real;
    using SH = Step2Shape<L, kF32>;
    if (!adjoint2_fits<L, S>(g)) return hipErrorInvalidValue;
    Step2Args aw, ar;
    aw.tiles_x = ar.tiles_x = g.nx / SH::TX;
    aw.tiles_y = ar.tiles_y = g.ny / SH::TY;
    aw.row_bytes = g.pitch * (uint32_t)sizeof(W);
    ar.row_bytes = g.pitch * (uint32_t)sizeof(R);
    aw.yrow_bytes = Lattice<L>::Q * aw.row_bytes;
    ar.yrow_bytes = Lattice<L>::Q * ar.row_bytes;
    aw.plane_bytes = g.ny * aw.yrow_bytes;
    ar.plane_bytes = g.ny * ar.yrow_bytes;
    const uint64_t tiles = (uint64_t)ar.tiles_x * ar.tiles_y;
    const uint32_t per_cu = force ? adjoint2_blocks_per_cu<L, S, true>() : adjoint2_blocks_per_cu<L, S, false>();
    ar.lz = aw.lz = step2_chunk(tiles, g.nz, (uint64_t)per_cu * device_cus(), 2);
    const dim3 grid((unsigned)(tiles * ((g.nz + ar.lz - 1) / ar.lz)));
    if (force)
      adjoint2_kernel<L, S, true><<<grid, SH::NT, 0, s>>>((const W*)gt, (const W*)gtm1, (const R*)chi_next,
                                                          (R*)chi_out, (const R*)force, (R*)dforce, g, aw, ar,
                                                          (R)omega);
    else
      adjoint2_kernel<L, S, false><<<grid, SH::NT, 0, s>>>((const W*)gt, (const W*)gtm1, (const R*)chi_next,
                                                           (R*)chi_out, nullptr, nullptr, g, aw, ar, (R)omega);
    return hipGetLastError();
  }
}

template <int L, int S>
static hipError_t launch_init_ls(const double* rho, const double* u, void* fout, const GridArgs& g, hipStream_t s) {
  using W = typename Storage<S>::word;
  init_kernel<L, S><<<cell_grid(g), 256, 0, s>>>(rho, u, (W*)fout, g);
  return hipGetLastError();
}

// Blocks of a moments launch whose blocks walk `span` blocks of cells each.
static uint64_t moments_blocks(const GridArgs& g, uint32_t span) { return (cell_grid(g).x + span - 1) / span; }

// Span of a reducing moments launch, measured: the fold costs about 150 VALU
// instructions per wave.  With fields stored, the 3D lattices are fastest at one cell per
// thread and D2Q9 (fewer loads per cell to hide the fold behind) at 4; with the
// reductions alone, at 16.
static uint32_t moments_span(int D, bool fields) { return fields ? (D == 2 ? 4 : 1) : 16; }

template <int L, int S, bool FORCED, uint32_t SPAN>
static void launch_moments_span(const typename Storage<S>::word* f, const typename Storage<S>::real* force,
                                typename Storage<S>::real* rho, typename Storage<S>::real* u, double* partials,
                                const GridArgs& g, hipStream_t s) {
  moments_kernel<L, S, FORCED, true, SPAN><<<(unsigned)moments_blocks(g, SPAN), 256,
                                             reserve_for_cap(moments_cap<L, S, FORCED, true, SPAN>()), s>>>(f, force, rho, u,
                                                                                             partials, g);
}

template <int L, int S>
static hipError_t launch_moments_ls(const void* f, const void* force, void* rho, void* u, double* workspace,
                                    double* red, const GridArgs& g, hipStream_t s) {
  using ST = Storage<S>;
  using W = typename ST::word;
  using R = typename ST::real;
  const W* fw = (const W*)f;
  const R* fr = (const R*)force;
  if (!red) {
    if (force)
      moments_kernel<L, S, true, false, 1><<<cell_grid(g), 256, reserve_for_cap(moments_cap<L, S, true, false, 1>()),
                                             s>>>(fw, fr, (R*)rho, (R*)u, nullptr, g);
    else
      moments_kernel<L, S, false, false, 1><<<cell_grid(g), 256, reserve_for_cap(moments_cap<L, S, false, false, 1>()),
                                              s>>>(fw, nullptr, (R*)rho, (R*)u, nullptr, g);
    return hipGetLastError();
  }
  const uint32_t span = moments_span(Lattice<L>::D, rho || u);
  const uint64_t p1 = moments_blocks(g, span);
  const uint64_t p2 = (p1 + kFoldBlock - 1) / kFoldBlock;
  double* part1 = workspace;
  double* part2 = workspace + p1 * kNred;
  R* rr = (R*)rho;
  R* ur = (R*)u;
  if (force) {
    if (span == 1) launch_moments_span<L, S, true, 1>(fw, fr, rr, ur, part1, g, s);
    if (span == 4) launch_moments_span<L, S, true, 4>(fw, fr, rr, ur, part1, g, s);
    if (span == 16) launch_moments_span<L, S, true, 16>(fw, fr, rr, ur, part1, g, s);
  } else {
    if (span == 1) launch_moments_span<L, S, false, 1>(fw, nullptr, rr, ur, part1, g, s);
    if (span == 4) launch_moments_span<L, S, false, 4>(fw, nullptr, rr, ur, part1, g, s);
    if (span == 16) launch_moments_span<L, S, false, 16>(fw, nullptr, rr, ur, part1, g, s);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  fold_partials_kernel<<<(unsigned)p2, 256, 0, s>>>(part1, p1, part2);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  reduce_partials_kernel<<<1, 256, 0, s>>>(part2, (int)p2, red, (double)g.ncells);
  return hipGetLastError();
}

template <int L, int S>
static hipError_t launch_moments_adjoint_ls(const void* f, const void* force, const void* drho, const void* du,
                                            void* lam_out, void* dforce, const GridArgs& g, hipStream_t s) {
  using ST = Storage<S>;
  using W = typename ST::word;
  using R = typename ST::real;
  moments_adjoint_kernel<L, S><<<cell_grid(g), 256, 0, s>>>((const W*)f, (const R*)force, (const R*)drho,
                                                             (const R*)du, (R*)lam_out, (R*)dforce, g);
  return hipGetLastError();
}

#define LBM_DISPATCH_STORAGE(LAUNCH, LAT, storage, ...)       \
  switch (storage) {                                         \
    case kF64: return LAUNCH<LAT, kF64>(__VA_ARGS__);        \
    case kF32: return LAUNCH<LAT, kF32>(__VA_ARGS__);        \
    case kF32S: return LAUNCH<LAT, kF32S>(__VA_ARGS__);      \
    case kF16S: return LAUNCH<LAT, kF16S>(__VA_ARGS__);      \
    case kBF16S: return LAUNCH<LAT, kBF16S>(__VA_ARGS__);    \
  }

#define LBM_DISPATCH(LAUNCH, lattice, storage, ...)                              \
  do {                                                                           \
    switch (lattice) {                                                           \
      case kD2Q9: LBM_DISPATCH_STORAGE(LAUNCH, kD2Q9, storage, __VA_ARGS__) break;   \
      case kD3Q19: LBM_DISPATCH_STORAGE(LAUNCH, kD3Q19, storage, __VA_ARGS__) break; \
      case kD3Q27: LBM_DISPATCH_STORAGE(LAUNCH, kD3Q27, storage, __VA_ARGS__) break; \
    }                                                                            \
    return hipErrorInvalidValue;                                                 \
  } while (0)

hipError_t launch_step(int lattice, int storage, const void* fin, void* fout, const void* force, int force_mode,
                       const GridArgs& g, double omega, hipStream_t s) {
  LBM_DISPATCH(launch_step_ls, lattice, storage, fin, fout, force, force_mode, g, omega, s);
}

int max_steps_per_launch(int lattice, int storage, const GridArgs& g) {
  int n = 1;
  auto check = [&]() -> hipError_t { LBM_DISPATCH(max_steps_ls, lattice, storage, g, &n); };
  return check() == hipSuccess ? n : 1;
}

hipError_t launch_stepn(int lattice, int storage, int nst, const void* fin, void* fout, const void* force,
                        int force_mode, const GridArgs& g, double omega, hipStream_t s) {
  LBM_DISPATCH(launch_stepn_ls, lattice, storage, nst, fin, fout, force, force_mode, g, omega, s);
}

bool step2_slab_supported(int lattice, int storage, const GridArgs& g) {
  bool ok = false;
  auto check = [&]() -> hipError_t { LBM_DISPATCH(step2_slab_fits_ls, lattice, storage, g, &ok); };
  return check() == hipSuccess && ok;
}

hipError_t launch_step2_slab(int lattice, int storage, const void* fin, void* fout, const void* force,
                             int force_mode, const GridArgs& g, double omega, hipStream_t s) {
  LBM_DISPATCH(launch_step2_slab_ls, lattice, storage, fin, fout, force, force_mode, g, omega, s);
}

bool adjoint2_supported(int lattice, int storage, const GridArgs& g) {
  bool ok = false;
  auto check = [&]() -> hipError_t { LBM_DISPATCH(adjoint2_fits_ls, lattice, storage, g, &ok); };
  return check() == hipSuccess && ok;
}

hipError_t launch_adjoint2(int lattice, int storage, const void* gt, const void* gtm1, const void* chi_next,
                           void* chi_out, const void* force, void* dforce, const GridArgs& g, double omega,
                           hipStream_t s) {
  LBM_DISPATCH(launch_adjoint2_ls, lattice, storage, gt, gtm1, chi_next, chi_out, force, dforce, g, omega, s);
}

hipError_t launch_adjoint(int lattice, int storage, int mode, const void* gt, const void* lam_next, void* lam_out,
                          const void* force, void* dforce, const GridArgs& g, double omega, hipStream_t s) {
  LBM_DISPATCH(launch_adjoint_ls, lattice, storage, mode, gt, lam_next, lam_out, force, dforce, g, omega, s);
}

hipError_t launch_init(int lattice, int storage, const double* rho, const double* u, void* fout, const GridArgs& g,
                       hipStream_t s) {
  LBM_DISPATCH(launch_init_ls, lattice, storage, rho, u, fout, g, s);
}

uint64_t moments_workspace_entries(const GridArgs& g) {
  const uint64_t p1 = moments_blocks(g, 1);  // the most partials of any span
  return p1 + (p1 + kFoldBlock - 1) / kFoldBlock;
}

uint64_t moments_entries_used(int lattice, const GridArgs& g, bool fields) {
  const uint64_t p1 = moments_blocks(g, moments_span(lattice == kD2Q9 ? 2 : 3, fields));
  return p1 + (p1 + kFoldBlock - 1) / kFoldBlock;
}

hipError_t launch_moments(int lattice, int storage, const void* f, const void* force, void* rho, void* u,
                          double* workspace, double* red, const GridArgs& g, hipStream_t s) {
  LBM_DISPATCH(launch_moments_ls, lattice, storage, f, force, rho, u, workspace, red, g, s);
}

hipError_t launch_moments_adjoint(int lattice, int storage, const void* f, const void* force, const void* drho,
                                  const void* du, void* lam_out, void* dforce, const GridArgs& g, hipStream_t s) {
  LBM_DISPATCH(launch_moments_adjoint_ls, lattice, storage, f, force, drho, du, lam_out, dforce, g, s);
}

template <int L>
static hipError_t launch_stream_l(int word_bytes, const void* fin, void* fout, const GridArgs& g, hipStream_t s) {
  switch (word_bytes) {
    case 2: stream_kernel<L, uint16_t><<<cell_grid(g), 256, 0, s>>>((const uint16_t*)fin, (uint16_t*)fout, g); break;
    case 4: stream_kernel<L, uint32_t><<<cell_grid(g), 256, 0, s>>>((const uint32_t*)fin, (uint32_t*)fout, g); break;
    case 8: stream_kernel<L, uint64_t><<<cell_grid(g), 256, 0, s>>>((const uint64_t*)fin, (uint64_t*)fout, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_stream(int lattice, int word_bytes, const void* fin, void* fout, const GridArgs& g, hipStream_t s) {
  switch (lattice) {
    case kD2Q9: return launch_stream_l<kD2Q9>(word_bytes, fin, fout, g, s);
    case kD3Q19: return launch_stream_l<kD3Q19>(word_bytes, fin, fout, g, s);
    case kD3Q27: return launch_stream_l<kD3Q27>(word_bytes, fin, fout, g, s);
  }
  return hipErrorInvalidValue;
}

// Plain streaming copy (16-byte words, one per thread, nontemporal loads and stores):
// the practical HBM bandwidth reference the step kernel is compared with.  Of the copy
// shapes measured (1, 2 or 4 words per thread, 256 or 512 threads, grid-stride loops,
// cached loads) this one moved the most bytes per second.

__global__ __launch_bounds__(256) void copy16_kernel(const u32x4* __restrict__ src, u32x4* __restrict__ dst, size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(&src[i]), &dst[i]);
}

hipError_t launch_copy16(const void* src, void* dst, size_t n16, hipStream_t s) {
  if (n16 == 0) return hipSuccess;
  copy16_kernel<<<(unsigned)((n16 + 255) / 256), 256, 0, s>>>((const u32x4*)src, (u32x4*)dst, n16);
  return hipGetLastError();
}

// z-slab halo exchange: direction rows [i0, i0 + n_dir) of each grid row of one plane,
// a contiguous chunk of n_dir * nx words per row at a pitch of Q * nx words.  T is the
// word type, or a 16-byte vector when nx words fill whole 16-byte units.
template <typename T>
__global__ __launch_bounds__(256) void halo_copy_kernel(const T* __restrict__ src, T* __restrict__ dst,
                                                        uint64_t src_base, uint64_t dst_base, uint64_t pitch,
                                                        uint64_t chunk, uint32_t ny) {
  const uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= chunk) return;
  for (uint32_t y = blockIdx.y; y < ny; y += gridDim.y) dst[dst_base + y * pitch + k] = src[src_base + y * pitch + k];
}

template <typename T>
static void launch_halo_t(const void* src, void* dst, uint64_t sb, uint64_t db, uint64_t pitch, uint64_t chunk,
                          uint32_t ny, hipStream_t s) {
  const dim3 grid((unsigned)((chunk + 255) / 256), ny < 4096u ? ny : 4096u);
  halo_copy_kernel<T><<<grid, 256, 0, s>>>((const T*)src, (T*)dst, sb, db, pitch, chunk, ny);
}

hipError_t launch_halo_copy(int Q, int word_bytes, const void* src, uint64_t src_plane, void* dst, uint64_t dst_plane,
                            int i0, int n_dir, uint32_t pitch, uint32_t ny, hipStream_t s) {
  const uint64_t row = (uint64_t)Q * pitch, chunk = (uint64_t)n_dir * pitch;
  const uint64_t sb = (src_plane * ny * Q + (uint64_t)i0) * pitch, db = (dst_plane * ny * Q + (uint64_t)i0) * pitch;
  if (((uint64_t)pitch * word_bytes) % 16 == 0) {  // every offset is a whole number of 16-byte units
    const uint64_t u = 16 / word_bytes;
    launch_halo_t<u32x4>(src, dst, sb / u, db / u, row / u, chunk / u, ny, s);
    return hipGetLastError();
  }
  switch (word_bytes) {
    case 2: launch_halo_t<uint16_t>(src, dst, sb, db, row, chunk, ny, s); break;
    case 4: launch_halo_t<uint32_t>(src, dst, sb, db, row, chunk, ny, s); break;
    case 8: launch_halo_t<uint64_t>(src, dst, sb, db, row, chunk, ny, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int L>
static hipError_t launch_unstream_l(int word_bytes, const void* fin, void* fout, const GridArgs& g, hipStream_t s) {
  switch (word_bytes) {
    case 4: unstream_kernel<L, uint32_t><<<cell_grid(g), 256, 0, s>>>((const uint32_t*)fin, (uint32_t*)fout, g); break;
    case 8: unstream_kernel<L, uint64_t><<<cell_grid(g), 256, 0, s>>>((const uint64_t*)fin, (uint64_t*)fout, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_unstream(int lattice, int word_bytes, const void* fin, void* fout, const GridArgs& g,
                           hipStream_t s) {
  switch (lattice) {
    case kD2Q9: return launch_unstream_l<kD2Q9>(word_bytes, fin, fout, g, s);
    case kD3Q19: return launch_unstream_l<kD3Q19>(word_bytes, fin, fout, g, s);
    case kD3Q27: return launch_unstream_l<kD3Q27>(word_bytes, fin, fout, g, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace lbm

// Device-side helpers shared by the kernel translation units: cell addressing in the
// row-interleaved population layout, the periodic (or ghost-plane) pull sources, and
// the BGK collision of one cell.
//
// Population layout ("row-interleaved SoA"): the grid is a set of rows r = z*ny + y of
// nx cells; row r stores its Q direction rows one after the other, so word (i, x) of
// row r sits at (r*Q + i)*nx + x.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "lattice.h"

namespace lbm {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));  // one 16-byte vector

__device__ __forceinline__ uint32_t wrap_dec(uint32_t v, uint32_t n) { return v == 0 ? n - 1 : v - 1; }
__device__ __forceinline__ uint32_t wrap_inc(uint32_t v, uint32_t n) { return v + 1 == n ? 0 : v + 1; }

template <typename T>
__device__ __forceinline__ void store_stream(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}

// A wave-uniform region [base, base + bytes) as a raw buffer resource (stride 0, no
// swizzle; word 3 is the gfx9 32-bit data format).  Loads and stores through it take
// the lane's 32-bit offset and a wave-uniform offset, so a run of accesses at uniform
// distances needs no per-access address arithmetic.  The hardware drops a store at or
// past `bytes` and returns 0 for such a load; the kernels keep every access inside.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t region_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// The T at byte voff + soff of a region (voff per lane, soff uniform); 0 at or past
// the region's end.
template <typename T>
__device__ __forceinline__ T region_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 2) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
  } else if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  } else {
    static_assert(sizeof(T) == 8, "2-, 4- or 8-byte words");
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  }
}

// Nontemporal store of v at byte voff + soff of a region (voff per lane, soff uniform).
template <typename T>
__device__ __forceinline__ void store_stream(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, T v) {
  constexpr int kNontemporal = 2;  // the cache-policy bit of a streaming store
  if constexpr (sizeof(T) == 2) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, voff, soff, kNontemporal);
  } else if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, kNontemporal);
  } else {
    static_assert(sizeof(T) == 8, "2-, 4- or 8-byte words");
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, kNontemporal);
  }
}

struct Cell {
  uint32_t x, y, z;
};

// The cell of a thread.  A 256-thread block covers block_x consecutive cells of
// 256/block_x consecutive rows; all 64 lanes of a wave share one row, so y and z are
// wave-uniform (made scalar with readfirstlane).  Returns false past the last row and
// for x >= x_end (nx for kernels that compute live cells only; the row pitch for the
// step, whose pad lanes store into the pad words).  `block` is the index of the block
// of cells, blockIdx.x unless a block walks several of them.
__device__ __forceinline__ bool cell_in_block(const GridArgs& g, Cell& c, uint32_t x_end, uint32_t block) {
  const uint32_t bx = g.block_x;
  const uint32_t blocks_x = (g.nx + bx - 1) / bx;
  const uint32_t bxi = block % blocks_x;
  const uint32_t byi = block / blocks_x;
  const uint32_t ty = __builtin_amdgcn_readfirstlane(threadIdx.x / bx);
  const uint32_t r = byi * (256u / bx) + ty;
  c.x = bxi * bx + threadIdx.x % bx;
  if (r >= g.ny * g.nzl) return false;
  c.y = r % g.ny;
  c.z = g.z0 + r / g.ny;
  return c.x < x_end;
}

__device__ __forceinline__ bool cell_below(const GridArgs& g, Cell& c, uint32_t x_end) {
  return cell_in_block(g, c, x_end, blockIdx.x);
}

__device__ __forceinline__ bool cell_of_thread(const GridArgs& g, Cell& c) { return cell_below(g, c, g.nx); }

// Source coordinates of the pull gather: index k = c + 1 holds the coordinate of
// x - c for c = -1, 0, +1, wrapped periodically (c = -1 reads x + 1).
struct Sources {
  uint32_t x[3];  // per lane
  uint32_t y[3];  // wave-uniform
  uint32_t z[3];  // wave-uniform
};

__device__ __forceinline__ Sources sources(const Cell& c, const GridArgs& g) {
  Sources s;
  s.x[0] = wrap_inc(c.x, g.nx);
  s.x[1] = c.x;
  s.x[2] = wrap_dec(c.x, g.nx);
  s.y[0] = wrap_inc(c.y, g.ny);
  s.y[1] = c.y;
  s.y[2] = wrap_dec(c.y, g.ny);
  if (g.ghost) {  // z-slab: neighbours in z are buffer planes c.z + 2 and c.z (ghost planes at the ends)
    s.z[0] = c.z + 2;
    s.z[1] = c.z + 1;
    s.z[2] = c.z;
  } else {
    s.z[0] = wrap_inc(c.z, g.nz);
    s.z[1] = c.z;
    s.z[2] = wrap_dec(c.z, g.nz);
  }
  return s;
}

// Word offset of direction row i of grid row (y, z): ((z*ny + y)*Q + i)*pitch.
template <int Q>
__device__ __forceinline__ uint64_t dir_row(const GridArgs& g, uint32_t y, uint32_t z, int i) {
  return (((uint64_t)z * g.ny + y) * Q + (uint64_t)i) * g.pitch;
}

// Word offset of the pull source of direction i for the cell: g_i(x - c_i).
template <typename LT>
__device__ __forceinline__ uint64_t src_offset(const GridArgs& g, const Sources& s, int i) {
  return dir_row<LT::Q>(g, s.y[LT::cy(i) + 1], s.z[LT::cz(i) + 1], i) + s.x[LT::cx(i) + 1];
}

// Word offset of direction i at x + c_i: the transpose of the pull gather (S^T).
template <typename LT>
__device__ __forceinline__ uint64_t rev_offset(const GridArgs& g, const Sources& s, int i) {
  return dir_row<LT::Q>(g, s.y[1 - LT::cy(i)], s.z[1 - LT::cz(i)], i) + s.x[1 - LT::cx(i)];
}

// Addressing split into a wave-uniform row base and a 32-bit per-lane byte offset: the
// row base lives in scalar registers and the compiler can use the scalar-base form of
// global loads and stores, with no per-lane 64-bit address arithmetic.
template <typename W>
__device__ __forceinline__ const W* at_byte(const W* row, uint32_t byte_offset) {
  return reinterpret_cast<const W*>(reinterpret_cast<const char*>(row) + byte_offset);
}
template <typename W>
__device__ __forceinline__ W* at_byte(W* row, uint32_t byte_offset) {
  return reinterpret_cast<W*>(reinterpret_cast<char*>(row) + byte_offset);
}

// The pull source g_i(x - c_i) of the cell, given the byte offsets xb[k] of the three
// source columns (k = c_x + 1 holds x - c_x).  8-byte words are loaded nontemporally:
// the FP64 steps ran 2% faster so (D3Q27 and D3Q19, three alternating A/B runs), while
// the same hint made the 2- and 4-byte steps 3-5% slower.
template <typename LT, typename W>
__device__ __forceinline__ W load_src(const W* f, const GridArgs& g, const Sources& s, const uint32_t (&xb)[3],
                                      int i) {
  const W* p = at_byte(f + dir_row<LT::Q>(g, s.y[LT::cy(i) + 1], s.z[LT::cz(i) + 1], i), xb[LT::cx(i) + 1]);
  if constexpr (sizeof(W) == 8)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

// The word of direction i at x + c_i (the transpose of the pull gather), same addressing.
template <typename LT, typename W>
__device__ __forceinline__ W load_rev(const W* f, const GridArgs& g, const Sources& s, const uint32_t (&xb)[3],
                                      int i) {
  return *at_byte(f + dir_row<LT::Q>(g, s.y[1 - LT::cy(i)], s.z[1 - LT::cz(i)], i), xb[1 - LT::cx(i)]);
}

// Byte offsets of the three source columns of a cell for words of type W.
template <typename W>
__device__ __forceinline__ void column_bytes(const Sources& s, uint32_t (&xb)[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) xb[k] = s.x[k] * (uint32_t)sizeof(W);
}

// acc += k * v for an integer lattice factor k in {-1, 0, 1}: an add, a subtract or
// nothing.  For finite v this equals the multiply-add bit for bit (one rounding of the
// exact sum, and 0 * v adds nothing), but the compiler may not drop a multiplication by
// 0.0 itself (it would change NaN and infinity propagation).
template <typename real>
__device__ __forceinline__ void add_times(real& acc, int k, real v) {
  if (k > 0) acc += v;
  if (k < 0) acc -= v;
}

// Linear cell index of real-valued fields ([D][N] arrays).
__device__ __forceinline__ uint32_t cell_index(const GridArgs& g, const Cell& c) {
  return (c.z * g.ny + c.y) * g.nx + c.x;
}


// ---------------------------------------------------------------------------------
// BGK collision of one cell in deviation form (Eqs. 2-4), in place: d holds the
// streamed populations h_i - w_i on entry and the post-collision deviations on exit.
// FM selects the per-cell field (Fx, Fy, Fz):
//   kNoForce     none
//   kGuoForce    body force F (Guo: u = (sum c h + F/2)/rho in f^eq, plus the source)
//   kShiftForce  velocity shift du: f^eq(rho, u + du) with u = sum c h / rho (the
//                flow-control forcing of Sec. 3.2)
//
// Products are fused into multiply-adds only within one expression (contract "on",
// not the default "fast", which lets the compiler fuse across statements depending on
// the code around the call): every kernel that inlines the collision then rounds
// identically, which the two-step kernel needs to reproduce two launches of the
// one-step kernel bit for bit.
// ---------------------------------------------------------------------------------
template <int L, typename real, int FM>
__device__ __forceinline__ void bgk_collide(real (&d)[Lattice<L>::Q], real Fx, real Fy, real Fz, real omega) {
#pragma clang fp contract(on)
  using LT = Lattice<L>;
  using CO = Coef<L, real>;
  constexpr int Q = LT::Q;
  constexpr bool D3 = LT::D == 3;
  // -0 is an exact additive identity (-0 + x == x for every x, signed zeros included),
  // so sums that start from it cost no instruction for their first term.
  constexpr real nzero = -0.0;
  // Moments (Eq. 4) in deviation form, rho = 1 + sum d, rho u = sum c d (+ F/2), from
  // partial sums: each row of velocities with equal (c_y, c_z) gives its sum and its
  // c_x-weighted sum, each plane of rows its sum and c_y-weighted sum.
  real drho = nzero, jx = nzero, jy = nzero, jz = nzero;
#pragma unroll
  for (int zc = (D3 ? -1 : 0); zc <= (D3 ? 1 : 0); ++zc) {
    real sp = nzero, yp = nzero;
#pragma unroll
    for (int yc = -1; yc <= 1; ++yc) {
      real sr = nzero, xr = nzero;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        if (LT::cy(i) != yc || LT::cz(i) != zc) continue;
        sr += d[i];
        if (LT::cx(i) > 0) xr += d[i];
        if (LT::cx(i) < 0) xr -= d[i];
      }
      sp += sr;
      if (yc > 0) yp += sr;
      if (yc < 0) yp -= sr;
      jx += xr;
    }
    drho += sp;
    jy += yp;
    if (zc > 0) jz += sp;
    if (zc < 0) jz -= sp;
  }
  constexpr bool FORCED = FM == kGuoForce;
  if constexpr (FORCED) {
    jx += real(0.5) * Fx;
    jy += real(0.5) * Fy;
    if constexpr (D3) jz += real(0.5) * Fz;
  }
  const real rho = real(1) + drho;
  const real inv_rho = real(1) / rho;
  real ux = jx * inv_rho, uy = jy * inv_rho, uz = 0;
  if constexpr (D3) uz = jz * inv_rho;
  if constexpr (FM == kShiftForce) {
    ux += Fx;
    uy += Fy;
    if constexpr (D3) uz += Fz;
  }
  const real usq = D3 ? real(1.5) * (ux * ux + uy * uy + uz * uz) : real(1.5) * (ux * ux + uy * uy);
  // Guo source G_i = (1 - omega/2) (A_i c_i.F - 3 W_i u.F + 2 B_i (c_i.u)(c_i.F)), with
  // the cell's factors taken out once: gF = (1 - omega/2) F, g3uF = 3 (1 - omega/2) u.F,
  // so that G_i = (c_i.gF)(A_i + 2 B_i c_i.u) - W_i g3uF
  const real guo = real(1) - real(0.5) * omega;
  const real gFx = guo * Fx, gFy = guo * Fy, gFz = guo * Fz;
  const real g3uF = D3 ? real(3) * (ux * gFx + uy * gFy + uz * gFz) : real(3) * (ux * gFx + uy * gFy);

  // c_i.u: computed for the first half of the velocities; the opposite velocity
  // (index Q-1-i in every lattice's order) takes its negation.
  real cuv[Q / 2];
#pragma unroll
  for (int i = 0; i < Q / 2; ++i) {
    real cu = nzero;
    if (LT::cx(i) > 0) cu += ux;
    if (LT::cx(i) < 0) cu -= ux;
    if (LT::cy(i) > 0) cu += uy;
    if (LT::cy(i) < 0) cu -= uy;
    if (LT::cz(i) > 0) cu += uz;
    if (LT::cz(i) < 0) cu -= uz;
    cuv[i] = cu;
  }
  // Equilibrium (Eq. 3) as a deviation,
  //   f^eq_i - w_i = W_i q + rho c.u (A_i + B_i c.u),   q = drho - rho usq,
  // and BGK relaxation (Eq. 2) as d + omega (deq - d): near equilibrium deq - d is
  // small and exact, which keeps the rounding of the relaxed value at half an ulp
  // (the equivalent (1 - omega) d + omega deq rounds twice on terms larger than the
  // result).  The class coefficients W_i, A_i, B_i enter only as factors of per-cell
  // values; a product of two run-wide constants (omega W_i, say) would carry one
  // rounding error into every collision and drift the momentum step after step.
  const real q = drho - rho * usq;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    constexpr real zero = 0;
    const real base = CO::W(i) * q;
    real deq = base;
    real cu = zero;
    if (LT::c2(i) != 0) {
      cu = i < Q / 2 ? cuv[i] : -cuv[Q - 1 - i];
      deq = rho * (cu * (CO::B(i) * cu + CO::A(i))) + base;
    }
    real dn = omega * (deq - d[i]) + d[i];
    if constexpr (FORCED) {
      real cgF = zero;
      add_times(cgF, LT::cx(i), gFx);
      add_times(cgF, LT::cy(i), gFy);
      add_times(cgF, LT::cz(i), gFz);
      dn += cgF * (CO::A(i) + real(2) * CO::B(i) * cu) - CO::W(i) * g3uF;
    }
    d[i] = dn;
  }
}

// ---------------------------------------------------------------------------------
// D2Q9 multiple-relaxation-time relaxation (Sec. 3.1, Eq. 5) in the Dellar basis, split
// so that the one-step and the multi-step kernels share it.  With the w-orthogonal
// rows R = {1, c_x, c_y, 3c_x^2-1, c_x c_y, 3c_y^2-1, g, g c_x, g c_y},
// g = (3c_x^2-1)(3c_y^2-1), the operator acting on h - f^eq is
//   f'_i = h_i - w_i sum_{k=3..8} R_k(c_i) s_k n_k,   n_k = sum_i R_k(c_i) (h_i - f^eq_i),
// s_k = 1/(tau_k |R_k|^2).  mrt_noneq takes the n_k of a cell's pulled deviations
// d = h - w, mrt_relax applies the update in place.  Products are fused only within an
// expression, so every kernel that inlines them rounds identically.
// ---------------------------------------------------------------------------------
template <typename real>
struct MrtScales {
  real s[6];  // s_3 .. s_8, rounded to the kernel's real type on the host
};

template <typename real>
struct MrtNoneq {
  real nxx, nxy, nyy, nN, nJx, nJy;  // n_3 .. n_8
};

template <typename real>
__device__ __forceinline__ MrtNoneq<real> mrt_noneq(const real (&d)[9]) {
#pragma clang fp contract(on)
  using LT = Lattice<kD2Q9>;
  // Raw moments of the deviations d = h - w; every R_k is orthogonal to w, so these are
  // the moments of h.  Lattice factors are 0, +-1, +-2 or 4: every product is exact.
  real drho = 0, jx = 0, jy = 0, sx = 0, sy = 0, pxy = 0, nN = 0, nJx = 0, nJy = 0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int cx = LT::cx(i), cy = LT::cy(i);
    drho += d[i];
    add_times(jx, cx, d[i]);
    add_times(jy, cy, d[i]);
    add_times(sx, cx * cx, d[i]);  // sum over c_x != 0
    add_times(sy, cy * cy, d[i]);
    add_times(pxy, cx * cy, d[i]);
    const real gd = real((3 * cx * cx - 1) * (3 * cy * cy - 1)) * d[i];
    nN += gd;
    add_times(nJx, cx, gd);
    add_times(nJy, cy, gd);
  }
  const real rho = real(1) + drho;
  const real inv_rho = real(1) / rho;
  const real ux = jx * inv_rho, uy = jy * inv_rho;
  // Subtract the moments of the second-order equilibrium, which have closed forms:
  // sum (3c_x^2 - 1) f^eq = 3 rho u_x^2, sum c_x c_y f^eq = rho u_x u_y, and the ghost
  // moments N, J of f^eq vanish.  sum (3c_x^2 - 1) d = 3 sx - drho.
  MrtNoneq<real> n;
  n.nxx = real(3) * sx - drho - real(3) * rho * ux * ux;
  n.nxy = pxy - rho * ux * uy;
  n.nyy = real(3) * sy - drho - real(3) * rho * uy * uy;
  n.nN = nN;
  n.nJx = nJx;
  n.nJy = nJy;
  return n;
}

// s: s_3 .. s_8 (the ghost scales s_6 .. s_8 uniform or the cell's own)
template <typename real>
__device__ __forceinline__ void mrt_relax(real (&d)[9], const MrtNoneq<real>& n, const real (&s)[6]) {
#pragma clang fp contract(on)
  using LT = Lattice<kD2Q9>;
  using CO = Coef<kD2Q9, real>;
  const real axx = n.nxx * s[0], axy = n.nxy * s[1], ayy = n.nyy * s[2];
  const real aN = n.nN * s[3], aJx = n.nJx * s[4], aJy = n.nJy * s[5];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int cx = LT::cx(i), cy = LT::cy(i);
    const real gi = real((3 * cx * cx - 1) * (3 * cy * cy - 1));
    real corr = real(3 * cx * cx - 1) * axx;
    add_times(corr, cx * cy, axy);
    corr += real(3 * cy * cy - 1) * ayy;
    real ghost_part = aN;
    add_times(ghost_part, cx, aJx);
    add_times(ghost_part, cy, aJy);
    corr += gi * ghost_part;
    d[i] = d[i] - CO::W(i) * corr;
  }
}

}  // namespace lbm

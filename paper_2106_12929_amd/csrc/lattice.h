// Compile-time lattice and storage descriptions shared by the HIP kernels.
//
// Velocity sets (paper Sec. 2.1, Eqs. 1-4, Sec. 3.3; textbook weights): D2Q9 and D3Q27
// are the tensor products of {-1, 0, 1}; direction i has c_x = i%3 - 1,
// c_y = (i/3)%3 - 1, c_z = i/9 - 1 (3D).  D3Q19 keeps the D3Q27 directions with
// |c|^2 <= 2, in the same order.  A weight depends on |c_i|^2 only.
// Every accessor is constexpr so that fully unrolled direction loops fold c_i and w_i
// into immediates.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "coeffs.h"

namespace lbm {

enum Lat { kD2Q9 = 0, kD3Q27 = 1, kD3Q19 = 2 };
enum Sto { kF64 = 0, kF32 = 1, kF32S = 2, kF16S = 3, kBF16S = 4 };

template <int L>
struct Lattice;

template <>
struct Lattice<kD2Q9> {
  static constexpr int D = 2;
  static constexpr int Q = 9;
  __host__ __device__ static constexpr int cx(int i) { return i % 3 - 1; }
  __host__ __device__ static constexpr int cy(int i) { return (i / 3) % 3 - 1; }
  __host__ __device__ static constexpr int cz(int) { return 0; }
  __host__ __device__ static constexpr int c2(int i) { return cx(i) * cx(i) + cy(i) * cy(i); }
  __host__ __device__ static constexpr double w(int i) {
    return (cx(i) * cx(i) + cy(i) * cy(i)) == 0 ? 4.0 / 9.0
         : (cx(i) * cx(i) + cy(i) * cy(i)) == 1 ? 1.0 / 9.0
                                                 : 1.0 / 36.0;
  }
};

template <>
struct Lattice<kD3Q27> {
  static constexpr int D = 3;
  static constexpr int Q = 27;
  __host__ __device__ static constexpr int cx(int i) { return i % 3 - 1; }
  __host__ __device__ static constexpr int cy(int i) { return (i / 3) % 3 - 1; }
  __host__ __device__ static constexpr int cz(int i) { return i / 9 - 1; }
  __host__ __device__ static constexpr int c2(int i) {
    return cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i);
  }
  __host__ __device__ static constexpr double w(int i) {
    return c2(i) == 0 ? 8.0 / 27.0 : c2(i) == 1 ? 2.0 / 27.0 : c2(i) == 2 ? 1.0 / 54.0 : 1.0 / 216.0;
  }
};

// D3Q27 index of each D3Q19 direction (the 8 corners |c|^2 = 3 left out).
constexpr int kD3Q19FromD3Q27[19] = {1, 3, 4, 5, 7, 9, 10, 11, 12, 13, 14, 15, 16, 17, 19, 21, 22, 23, 25};

template <>
struct Lattice<kD3Q19> {
  static constexpr int D = 3;
  static constexpr int Q = 19;
  __host__ __device__ static constexpr int cx(int i) { return kD3Q19FromD3Q27[i] % 3 - 1; }
  __host__ __device__ static constexpr int cy(int i) { return (kD3Q19FromD3Q27[i] / 3) % 3 - 1; }
  __host__ __device__ static constexpr int cz(int i) { return kD3Q19FromD3Q27[i] / 9 - 1; }
  __host__ __device__ static constexpr int c2(int i) {
    return cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i);
  }
  __host__ __device__ static constexpr double w(int i) {
    return c2(i) == 0 ? 1.0 / 3.0 : c2(i) == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
  }
};

// ---------------------------------------------------------------------------------
// Equilibrium coefficients in the working precision R:
//   deq_i = W_i drho + rho (A_i (c_i.u) + B_i (c_i.u)^2 - W_i 3/2 |u|^2)
// Nominally W = w, A = 3 w, B = 9/2 w (Eq. 3, c_s^2 = 1/3).  In FP32 the class values
// come from coeffs.h, chosen so that the mass and momentum sums are exact on the
// binary32 values (otherwise every step rescales the momentum by ~1 + 1e-8).
// ---------------------------------------------------------------------------------
template <int L, typename R>
struct Coef;

template <int L>
struct Coef<L, double> {
  __host__ __device__ static constexpr double W(int i) { return Lattice<L>::w(i); }
  __host__ __device__ static constexpr double A(int i) { return 3.0 * Lattice<L>::w(i); }
  __host__ __device__ static constexpr double B(int i) { return 4.5 * Lattice<L>::w(i); }
};

template <>
struct Coef<kD2Q9, float> {
  using LT = Lattice<kD2Q9>;
  __host__ __device__ static constexpr float W(int i) { return kD2Q9_W[LT::c2(i)]; }
  __host__ __device__ static constexpr float A(int i) { return kD2Q9_A[LT::c2(i)]; }
  __host__ __device__ static constexpr float B(int i) { return kD2Q9_B[LT::c2(i)]; }
};

template <>
struct Coef<kD3Q19, float> {
  using LT = Lattice<kD3Q19>;
  __host__ __device__ static constexpr float W(int i) { return kD3Q19_W[LT::c2(i)]; }
  __host__ __device__ static constexpr float A(int i) { return kD3Q19_A[LT::c2(i)]; }
  __host__ __device__ static constexpr float B(int i) { return kD3Q19_B[LT::c2(i)]; }
};

template <>
struct Coef<kD3Q27, float> {
  using LT = Lattice<kD3Q27>;
  __host__ __device__ static constexpr float W(int i) { return kD3Q27_W[LT::c2(i)]; }
  __host__ __device__ static constexpr float A(int i) { return kD3Q27_A[LT::c2(i)]; }
  __host__ __device__ static constexpr float B(int i) { return kD3Q27_B[LT::c2(i)]; }
};

// ---------------------------------------------------------------------------------
// Rounding helpers (IEEE round to nearest even, subnormals kept).
// ---------------------------------------------------------------------------------

__device__ __forceinline__ uint16_t f32_to_f16_bits(float x) {
  _Float16 h = static_cast<_Float16>(x);  // v_cvt_f16_f32: RNE in the default mode
  return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_bits_to_f32(uint16_t b) {
  return static_cast<float>(__builtin_bit_cast(_Float16, b));
}
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float x) {
  __bf16 h = static_cast<__bf16>(x);  // v_cvt_pk_bf16_f32: RNE; a NaN stays a (quiet) NaN
  return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) {
  return __builtin_bit_cast(float, static_cast<uint32_t>(b) << 16);
}
// double -> float rounded toward zero with a sticky last bit ("round to odd").  A
// following RNE conversion to a format with at most 24-2 = 22 significand bits then
// gives the correctly rounded double -> narrow result (no double-rounding error).
__device__ __forceinline__ float f64_to_f32_odd(double d) {
  float f = static_cast<float>(d);
  if (static_cast<double>(f) == d) return f;
  uint32_t b = __builtin_bit_cast(uint32_t, f);
  if (fabs(static_cast<double>(f)) > fabs(d)) b -= 1u;  // step back toward zero
  return __builtin_bit_cast(float, b | 1u);
}

// ---------------------------------------------------------------------------------
// Storage kinds.  to_dev(word, w) returns the deviation d = f - w in the working
// precision; from_dev(d, w) returns the word to store for f = w + d.
// ---------------------------------------------------------------------------------

template <int S>
struct Storage;

template <>
struct Storage<kF64> {
  using word = double;
  using real = double;
  __device__ static real to_dev(word v, real w) { return v - w; }
  __device__ static word from_dev(real d, real w) { return w + d; }
  __device__ static word from_f64_dev(double d, double w) { return w + d; }
};

template <>
struct Storage<kF32> {
  using word = float;
  using real = float;
  __device__ static real to_dev(word v, real w) { return v - w; }
  __device__ static word from_dev(real d, real w) { return w + d; }
  __device__ static word from_f64_dev(double d, double w) { return static_cast<float>(w + d); }
};

template <>
struct Storage<kF32S> {
  using word = float;
  using real = float;
  __device__ static real to_dev(word v, real) { return v; }
  __device__ static word from_dev(real d, real) { return d; }
  __device__ static word from_f64_dev(double d, double) { return static_cast<float>(d); }
};

template <>
struct Storage<kF16S> {
  using word = uint16_t;
  using real = float;
  __device__ static real to_dev(word v, real) { return f16_bits_to_f32(v); }
  __device__ static word from_dev(real d, real) { return f32_to_f16_bits(d); }
  __device__ static word from_f64_dev(double d, double) { return f32_to_f16_bits(f64_to_f32_odd(d)); }
};

template <>
struct Storage<kBF16S> {
  using word = uint16_t;
  using real = float;
  __device__ static real to_dev(word v, real) { return bf16_bits_to_f32(v); }
  __device__ static word from_dev(real d, real) { return f32_to_bf16_bits(d); }
  __device__ static word from_f64_dev(double d, double) { return f32_to_bf16_bits(f64_to_f32_odd(d)); }
};

}  // namespace lbm

// Device arithmetic helpers for double and interleaved complex double.
#pragma once
#include <hip/hip_runtime.h>

#include "fa_internal.hpp"

namespace fa {

__device__ __forceinline__ double zero(double) { return 0.0; }
__device__ __forceinline__ cplx zero(cplx) { return cplx{0.0, 0.0}; }

__device__ __forceinline__ cplx operator+(cplx a, cplx b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cplx operator-(cplx a, cplx b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cplx operator*(cplx a, cplx b) {
  return {fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x)};
}
__device__ __forceinline__ cplx operator*(double a, cplx b) { return {a * b.x, a * b.y}; }
__device__ __forceinline__ cplx& operator+=(cplx& a, cplx b) { a.x += b.x; a.y += b.y; return a; }
__device__ __forceinline__ cplx& operator-=(cplx& a, cplx b) { a.x -= b.x; a.y -= b.y; return a; }

// a * b + c
__device__ __forceinline__ double mad(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ cplx mad(cplx a, cplx b, cplx c) {
  return {fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y))};
}
// conj(a) * b + c
__device__ __forceinline__ double cmad(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ cplx cmad(cplx a, cplx b, cplx c) {
  return {fma(a.x, b.x, fma(a.y, b.y, c.x)), fma(a.x, b.y, fma(-a.y, b.x, c.y))};
}
__device__ __forceinline__ bool is_zero(double a) { return a == 0.0; }
__device__ __forceinline__ bool is_zero(cplx a) { return a.x == 0.0 && a.y == 0.0; }
__device__ __forceinline__ double abs2(double a) { return a * a; }
__device__ __forceinline__ double abs2(cplx a) { return fma(a.x, a.x, a.y * a.y); }
__device__ __forceinline__ cplx times_i(cplx a) { return {-a.y, a.x}; }   //  i a
__device__ __forceinline__ cplx times_mi(cplx a) { return {a.y, -a.x}; }  // -i a
__device__ __forceinline__ cplx conjg(cplx a) { return {a.x, -a.y}; }

__device__ __forceinline__ double shfl_xor(double v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ cplx shfl_xor(cplx v, int m) {
  return {__shfl_xor(v.x, m, 64), __shfl_xor(v.y, m, 64)};
}
__device__ __forceinline__ double shfl_down(double v, int d, int w) { return __shfl_down(v, d, w); }
__device__ __forceinline__ cplx shfl_down(cplx v, int d, int w) {
  return {__shfl_down(v.x, d, w), __shfl_down(v.y, d, w)};
}

// sum over the 64 lanes of a wavefront, same value in every lane, fixed order
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += shfl_xor(v, m);
  return v;
}

// Workgroup index remap for the 8 XCDs of the chip: the hardware hands
// consecutive workgroups to the XCDs in turn, so logical tile
// xcd_contiguous(b) gives each XCD one contiguous range of tiles (neighbouring
// tiles share halos in that XCD's L2).
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_contiguous(int bid, int nwg) {
  const int per = nwg / kXcds, rem = nwg % kXcds;
  const int xcd = bid % kXcds, k = bid / kXcds;
  return (xcd < rem) ? xcd * (per + 1) + k : rem * (per + 1) + (xcd - rem) * per + k;
}

template <typename T> struct host_to_dev;
template <> struct host_to_dev<double> {
  static double conv(const cd& z) { return z.real(); }
};
template <> struct host_to_dev<cplx> {
  static cplx conv(const cd& z) { return cplx{z.real(), z.imag()}; }
};

}  // namespace fa

// Complex helpers for the gfx950 kernels: interleaved (re, im) values held in
// float2 / double2, and 16-byte "packs" (float4 = two complex64, double2 = one
// complex128) used for coalesced vector loads.
#pragma once
#include <hip/hip_runtime.h>

namespace tuckfmm {

template <typename T> struct Tr;
template <> struct Tr<float> {
  using c = float2;
  using pack = float4;
  static constexpr int E = 2;  // complex values per 16-byte pack
};
template <> struct Tr<double> {
  using c = double2;
  using pack = double2;
  static constexpr int E = 1;
};

__host__ __device__ constexpr int round_up(int v, int m) { return (v + m - 1) / m * m; }

// acc += a * b
__device__ __forceinline__ void cfma(float2& acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(-a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(a.y, b.x, acc.y);
}
__device__ __forceinline__ void cfma(double2& acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
__device__ __forceinline__ void cfma_conj(float2& acc, float2 a, float2 b) {
  acc.x = fmaf(a.x, b.x, acc.x);
  acc.x = fmaf(a.y, b.y, acc.x);
  acc.y = fmaf(a.x, b.y, acc.y);
  acc.y = fmaf(-a.y, b.x, acc.y);
}
__device__ __forceinline__ void cfma_conj(double2& acc, double2 a, double2 b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}

// acc += sum over the pack of a_k * b_k (complex)
__device__ __forceinline__ void pdot(float2& acc, float4 a, float4 b) {
  cfma(acc, make_float2(a.x, a.y), make_float2(b.x, b.y));
  cfma(acc, make_float2(a.z, a.w), make_float2(b.z, b.w));
}
__device__ __forceinline__ void pdot(double2& acc, double2 a, double2 b) { cfma(acc, a, b); }

// o_k += a_k * s for every complex value of the pack
__device__ __forceinline__ void paxpy(float4& o, float4 a, float2 s) {
  o.x = fmaf(a.x, s.x, o.x);
  o.x = fmaf(-a.y, s.y, o.x);
  o.y = fmaf(a.x, s.y, o.y);
  o.y = fmaf(a.y, s.x, o.y);
  o.z = fmaf(a.z, s.x, o.z);
  o.z = fmaf(-a.w, s.y, o.z);
  o.w = fmaf(a.z, s.y, o.w);
  o.w = fmaf(a.w, s.x, o.w);
}
__device__ __forceinline__ void paxpy(double2& o, double2 a, double2 s) { cfma(o, a, s); }

__device__ __forceinline__ float4 padd(float4 a, float4 b) {
  return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}
__device__ __forceinline__ double2 padd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

template <typename P> __device__ __forceinline__ P pzero();
template <> __device__ __forceinline__ float4 pzero<float4>() { return make_float4(0.f, 0.f, 0.f, 0.f); }
template <> __device__ __forceinline__ double2 pzero<double2>() { return make_double2(0.0, 0.0); }

template <typename C> __device__ __forceinline__ C czero();
template <> __device__ __forceinline__ float2 czero<float2>() { return make_float2(0.f, 0.f); }
template <> __device__ __forceinline__ double2 czero<double2>() { return make_double2(0.0, 0.0); }

__device__ __forceinline__ float2 conjc(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ double2 conjc(double2 a) { return make_double2(a.x, -a.y); }

// Sum over the 64 lanes of a wavefront; every lane receives the total.
template <typename C> __device__ __forceinline__ C wave_sum(C v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v.x += __shfl_xor(v.x, o, 64);
    v.y += __shfl_xor(v.y, o, 64);
  }
  return v;
}

}  // namespace tuckfmm

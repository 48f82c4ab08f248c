// quad4.h -- 4x4 block rows spread over a quad of lanes (lane `row` of a
// cell holds one block row and one entry of each 4-vector), shared by the
// second-stage sweeps.  Include inside an anonymous namespace.
#pragma once
#include <hip/hip_runtime.h>

// value of lane M of the quad, in every lane of the quad (DPP quad_perm)
template <int M> __device__ __forceinline__ float qb(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), M | (M << 2) | (M << 4) | (M << 6), 0xf, 0xf, true));
}
template <int M> __device__ __forceinline__ double qb(double v) {
  long long u = __double_as_longlong(v);
  int lo = __builtin_amdgcn_mov_dpp((int)(u & 0xffffffff), M | (M << 2) | (M << 4) | (M << 6), 0xf, 0xf, true);
  int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), M | (M << 2) | (M << 4) | (M << 6), 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// (M v)[row] for the 4-vector v spread over the quad (lane m holds v[m]);
// every lane of the quad must be active
template <class T> __device__ __forceinline__ T quad_mv(const T (&Mrow)[4], T v) {
  T o = Mrow[0] * qb<0>(v);
  o = fma(Mrow[1], qb<1>(v), o);
  o = fma(Mrow[2], qb<2>(v), o);
  o = fma(Mrow[3], qb<3>(v), o);
  return o;
}

template <class T>
__device__ __forceinline__ T dot4(const T *__restrict__ a, const T (&y)[4]) {
  T u = 0;
#pragma unroll
  for (int m = 0; m < 4; ++m) u = fma(a[m], y[m], u);
  return u;
}

template <class T> __device__ __forceinline__ void ld4(const T *p, T (&o)[4]) {
#pragma unroll
  for (int m = 0; m < 4; ++m) o[m] = p[m];
}
// 4 consecutive values in 16-byte loads (p 16-byte aligned)
__device__ __forceinline__ void ld4v(const float *p, float (&o)[4]) {
  float4 a = *(const float4 *)p;
  o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
}
__device__ __forceinline__ void ld4v(const double *p, double (&o)[4]) {
  double2 a = ((const double2 *)p)[0], b2 = ((const double2 *)p)[1];
  o[0] = a.x; o[1] = a.y; o[2] = b2.x; o[3] = b2.y;
}
// 8 consecutive values (p aligned to 16 bytes)
__device__ __forceinline__ void ld8v(const float *p, float (&o)[8]) {
  float4 a = ((const float4 *)p)[0], b2 = ((const float4 *)p)[1];
  o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w; o[4] = b2.x; o[5] = b2.y; o[6] = b2.z; o[7] = b2.w;
}
__device__ __forceinline__ void ld8v(const double *p, double (&o)[8]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) { double2 a = ((const double2 *)p)[q]; o[2 * q] = a.x; o[2 * q + 1] = a.y; }
}

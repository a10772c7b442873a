// nesting_kernels.hip -- sampled sup |f_a - f_b| over a box (two levels, or a
// level and a reference shape's SDF), the quantity the paper's Propositions
// 1-2 turn into nesting thresholds (Sec. 3.3: the infinity norm on the
// training domain, approximated by a maximum over sampled points).
//
// Points come from a counter-based generator so that any other implementation
// can reproduce them exactly: splitmix64 (Steele, Lea and Flood, 2014, with
// Vigna's published finaliser), stream position k = 4 i + c for coordinate c of
// point i, u = top 24 bits / 2^24, x_c = float(lo + (hi - lo) u) evaluated in
// double (one rounding), and the time coordinate t = u of c = 3.
#include "nnm_kernels.h"

namespace nnm {

__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
  uint64_t z = seed + (k + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_box_points(uint64_t seed, long long base, int count, float lo, float hi, float* x, float* t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const uint64_t p = (uint64_t)(base + i);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double u = (double)(splitmix64_at(seed, 4ull * p + c) >> 40) * (1.0 / 16777216.0);
    x[3 * i + c] = (float)((double)lo + ((double)hi - (double)lo) * u);
  }
  if (t) t[i] = (float)((double)(splitmix64_at(seed, 4ull * p + 3) >> 40) * (1.0 / 16777216.0));
}

// Non-negative floats order like their bit patterns, so the maximum is an
// unsigned atomicMax; a NaN difference counts as +inf.
__global__ void k_absdiff_max(const float* fa, const float* fb, int count, unsigned int* out) {
  __shared__ float red[256];
  float m = 0.f;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    float d = fabsf(fa[i] - fb[i]);
    if (!(d >= 0.f)) d = __builtin_inff();
    m = fmaxf(m, d);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, __float_as_uint(red[0]));
}

// Signed distance of a reference shape at points x[count][3], in float32:
// kind 1 sphere |x| - a; kind 2 torus about the z axis with major radius a and
// minor radius b, sqrt((sqrt(x^2 + y^2) - a)^2 + z^2) - b.
__global__ void k_ref_sdf(const float* x, int count, int kind, float a, float b, float* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float px = x[3 * i], py = x[3 * i + 1], pz = x[3 * i + 2];
  float d;
  if (kind == 1) {
    d = sqrtf(fmaf(px, px, fmaf(py, py, pz * pz))) - a;
  } else {
    const float q = sqrtf(fmaf(px, px, py * py)) - a;
    d = sqrtf(fmaf(q, q, pz * pz)) - b;
  }
  out[i] = d;
}

hipError_t launch_ref_sdf(const float* x, int count, int kind, float a, float b, float* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ref_sdf, dim3((count + 255) / 256), dim3(256), 0, s, x, count, kind, a, b, out);
  return hipGetLastError();
}

hipError_t launch_box_points(uint64_t seed, long long base, int count, float lo, float hi, float* x, float* t,
                             hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_box_points, dim3((count + 255) / 256), dim3(256), 0, s, seed, base, count, lo, hi, x, t);
  return hipGetLastError();
}

hipError_t launch_absdiff_max(const float* fa, const float* fb, int count, unsigned int* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const int grid = std::min(2048, (count + 255) / 256);
  hipLaunchKernelGGL(k_absdiff_max, dim3(grid), dim3(256), 0, s, fa, fb, count, out);
  return hipGetLastError();
}

}  // namespace nnm

// Colour front end on gfx950: 8-bit sRGB to CIELAB (the paper works in
// CIELAB, Sec. IV).  sRGB per IEC 61966-2-1, the sRGB primaries with the D65
// white, CIE 1976 L*a*b* relative to D65 (2-degree observer).
//
// Memory-bound: 3 bytes in, 12 bytes out per pixel.  Each thread converts four
// pixels (one 12-byte read); the block's results are staged in LDS and written
// as contiguous 16-byte spans per instruction; the 256-entry transfer
// function is tabulated per block in LDS (FP64, rounded once to FP32), so a
// pixel costs three LDS reads, nine FMAs and three cube roots (three
// transcendental instructions and a Newton step each).
#include "gmmsp_internal.h"

#include <math.h>

namespace gmmsp {

namespace {

constexpr int kT = 256;

// linear RGB -> (X / X_n, Y / Y_n, Z / Z_n): the sRGB primaries' matrix with
// each row divided by the D65 white
__device__ __constant__ float kM[9] = {
    0.4124564f / 0.95047f, 0.3575761f / 0.95047f, 0.1804375f / 0.95047f,
    0.2126729f, 0.7151522f, 0.0721750f,
    0.0193339f / 1.08883f, 0.1191920f / 1.08883f, 0.9503041f / 1.08883f};

// t^(1/3) for t > (6/29)^3: exp2(log2(t) / 3) (relative error a few 1e-7),
// then one Newton step y <- y + (t / y^2 - y) / 3, which squares the error
__device__ __forceinline__ float cube_root(float t) {
  const float y = __builtin_amdgcn_exp2f(__builtin_amdgcn_logf(t) * (1.0f / 3.0f));
  const float r = __builtin_amdgcn_rcpf(y);
  return fmaf(fmaf(t * r, r, -y), 1.0f / 3.0f, y);
}

__device__ __forceinline__ float lab_f(float t) {
  constexpr float d3 = (6.0f / 29.0f) * (6.0f / 29.0f) * (6.0f / 29.0f);
  constexpr float k = 1.0f / (3.0f * (6.0f / 29.0f) * (6.0f / 29.0f));
  return t > d3 ? cube_root(t) : fmaf(t, k, 4.0f / 29.0f);
}

__device__ __forceinline__ void convert(const float* lut, uint32_t r, uint32_t g, uint32_t b,
                                        float* out) {
  const float lr = lut[r], lg = lut[g], lb = lut[b];
  const float x = fmaf(kM[0], lr, fmaf(kM[1], lg, kM[2] * lb));
  const float y = fmaf(kM[3], lr, fmaf(kM[4], lg, kM[5] * lb));
  const float z = fmaf(kM[6], lr, fmaf(kM[7], lg, kM[8] * lb));
  const float fx = lab_f(x), fy = lab_f(y), fz = lab_f(z);
  out[0] = fmaf(116.0f, fy, -16.0f);
  out[1] = 500.0f * (fx - fy);
  out[2] = 200.0f * (fy - fz);
}

__global__ __launch_bounds__(kT) void k_srgb8_to_lab(const uint8_t* __restrict__ rgb, int64_t n,
                                                     float* __restrict__ lab) {
  __shared__ float lut[256];
  __shared__ float4 stage[3 * kT];  // the block's 4 kT pixels of output
  {
    const double c = threadIdx.x / 255.0;
    lut[threadIdx.x] = (float)(c <= 0.04045 ? c / 12.92 : pow((c + 0.055) / 1.055, 2.4));
  }
  __syncthreads();
  const int64_t groups = n / 4;            // four pixels per thread
  const int64_t tiles = groups / kT;       // whole blocks of 4 kT pixels
  for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const int64_t q = tile * kT + threadIdx.x;
    const uint3 w = *reinterpret_cast<const uint3*>(rgb + 12 * q);
    const uint32_t v[3] = {w.x, w.y, w.z};
    float o[12];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      uint32_t c[3];
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        const int byte = 3 * p + ch;
        c[ch] = (v[byte >> 2] >> (8 * (byte & 3))) & 0xFFu;
      }
      convert(lut, c[0], c[1], c[2], o + 3 * p);
    }
    // through LDS, so that each store instruction writes one contiguous span
    stage[3 * threadIdx.x + 0] = make_float4(o[0], o[1], o[2], o[3]);
    stage[3 * threadIdx.x + 1] = make_float4(o[4], o[5], o[6], o[7]);
    stage[3 * threadIdx.x + 2] = make_float4(o[8], o[9], o[10], o[11]);
    __syncthreads();
    float4* dst = reinterpret_cast<float4*>(lab + 12 * tile * kT);
#pragma unroll
    for (int k = 0; k < 3; ++k) dst[k * kT + threadIdx.x] = stage[k * kT + threadIdx.x];
    __syncthreads();
  }
  // the pixels after the last whole block, one per thread of block 0
  if (blockIdx.x == 0) {
    for (int64_t i = 4 * tiles * kT + threadIdx.x; i < n; i += kT)
      convert(lut, rgb[3 * i], rgb[3 * i + 1], rgb[3 * i + 2], lab + 3 * i);
  }
}

}  // namespace

hipError_t launch_srgb8_to_lab(const uint8_t* rgb, int64_t n, float* lab, hipStream_t s) {
  int64_t blocks = n / (4 * kT);
  if (blocks > 8192) blocks = 8192;  // grid-stride beyond 32 blocks per CU
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_srgb8_to_lab, dim3((unsigned)blocks), dim3(kT), 0, s, rgb, n, lab);
  return hipGetLastError();
}

}  // namespace gmmsp

// Device helpers shared by the per-cell kernels (gmmsp_kernels.hip,
// gmmsp_cov3.hip, gmmsp_modes.hip): scalar-load pointers, FP64 constants and
// the wave-wide butterfly reduce-scatter.  Not part of the public ABI.
#pragma once

#include "gmmsp_internal.h"

namespace gmmsp {

#define AS4 __attribute__((address_space(4)))

// Uniform reads through the constant address space compile to scalar loads.
template <typename T>
__device__ __forceinline__ const AS4 T* cptr(const T* p) {
  return (const AS4 T*)(p);
}

constexpr double kLog2e = 1.4426950408889634074;
constexpr double kLn2 = 0.69314718055994530942;
constexpr double kLn2Pi = 1.8378770664093454836;

// Butterfly reduce-scatter of per-lane sums across a 64-lane wave.  Each step
// halves the number of values: in a pair of partner lanes the one whose keep
// bit is 0 keeps the even entries summed with its partner's, the other the odd
// ones.  Keep bits go 5, 4, 3, 2, 1, 0: each step consumes the lowest bit of an
// entry's index, so after the six steps lane l holds the wave total of entry
// 64 q + bitrev6(l) at position q.

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// keep bit 5 (lanes 0-31 keep even entries): v_permlane32_swap exchanges the
// upper half of the first operand with the lower half of the second.
template <int N, int CAP>
__device__ __forceinline__ void bfly_swap32(float (&v)[CAP]) {
  static_assert(2 * ((N + 1) / 2) <= CAP, "butterfly reads past the array");
  if (N & 1) v[N] = 0.f;
#pragma unroll
  for (int i = 0; i < (N + 1) / 2; ++i) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[2 * i]),
                                                    __float_as_uint(v[2 * i + 1]), false, false);
    v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
}

// keep bit 4: v_permlane16_swap exchanges odd 16-lane rows of the first operand
// with even rows of the second.
template <int N, int CAP>
__device__ __forceinline__ void bfly_swap16(float (&v)[CAP]) {
  static_assert(2 * ((N + 1) / 2) <= CAP, "butterfly reads past the array");
  if (N & 1) v[N] = 0.f;
#pragma unroll
  for (int i = 0; i < (N + 1) / 2; ++i) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[2 * i]),
                                                    __float_as_uint(v[2 * i + 1]), false, false);
    v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
}

// keep bit BIT, partner given by the DPP control CTRL (an involution inside a
// 16-lane row that flips BIT and keeps the higher bits)
template <int N, int BIT, int CTRL, int CAP>
__device__ __forceinline__ void bfly_dpp(float (&v)[CAP], int lane) {
  static_assert(2 * ((N + 1) / 2) <= CAP, "butterfly reads past the array");
  const bool hi = ((lane >> BIT) & 1) != 0;
  if (N & 1) v[N] = 0.f;
#pragma unroll
  for (int i = 0; i < (N + 1) / 2; ++i) {
    const float a = v[2 * i], b = v[2 * i + 1];
    const float send = hi ? a : b;
    const float keep = hi ? b : a;
    v[i] = keep + dpp<CTRL>(send);
  }
}

// N per-lane values (the array holds at least 2 ceil(N / 2)); afterwards lane
// l holds the wave total of entry 64 q + bitrev6(l) in v[q].
template <int N, int CAP>
__device__ __forceinline__ void wave_reduce_scatter(float (&v)[CAP], int lane) {
  constexpr int N1 = (N + 1) / 2, N2 = (N1 + 1) / 2, N3 = (N2 + 1) / 2, N4 = (N3 + 1) / 2,
                N5 = (N4 + 1) / 2;
  bfly_swap32<N>(v);
  bfly_swap16<N1>(v);
  bfly_dpp<N2, 3, 0x128>(v, lane);  // row_ror:8, partner lane ^ 8
  bfly_dpp<N3, 2, 0x141>(v, lane);  // row_half_mirror, partner lane ^ 7
  bfly_dpp<N4, 1, 0x4E>(v, lane);   // quad_perm [2,3,0,1], partner lane ^ 2
  bfly_dpp<N5, 0, 0xB1>(v, lane);   // quad_perm [1,0,3,2], partner lane ^ 1
}

// ---------------------------------------------------------------------------
// Record offsets through LDS.  A VALU FMA reads at most one scalar register, so
// the offset of a whitening FMA (the addend beside a scalar record factor) has
// to come from a vector register.  The per-cell kernels keep the nine slots'
// offsets (at most 5 per record) in the wave's own block of LDS, kOffStride
// floats per slot, and read them back by broadcast each round: LDS reads issue
// on their own port, so this costs no VALU issue and no scalar registers.
// ---------------------------------------------------------------------------
constexpr int kOffStride = 8;
constexpr int kOffBlock = kSlots * kOffStride;  // floats per wave

// lanes 0..kSlots-1 copy the offsets idx[0..N) of their slot's record (rec_cell:
// the cell's slot-0 record, slot s at s * rec_stride floats); every lane of the wave may read the
// block after the call.  Only the calling wave touches its block, so a wave
// barrier orders the writes before the reads.
template <int N>
__device__ __forceinline__ void stage_offsets(float* woff, const float* rec_cell, size_t rec_stride,
                                              const int (&idx)[N], int lane) {
  static_assert(N <= 5, "at most five offsets per record");
  if (lane < kSlots) {
    const float* g = rec_cell + (size_t)lane * rec_stride;
#pragma unroll
    for (int i = 0; i < N; ++i) woff[lane * kOffStride + i] = g[idx[i]];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// the offsets of slot s: four by one 16-byte read, the fifth by one more
template <int N>
__device__ __forceinline__ void load_offsets(const float* woff, int s, float (&o)[N]) {
  const float4 q = *reinterpret_cast<const float4*>(woff + s * kOffStride);
  const float v[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
  for (int i = 0; i < N && i < 4; ++i) o[i] = v[i];
  if constexpr (N > 4) o[4] = woff[s * kOffStride + 4];
}

}  // namespace gmmsp

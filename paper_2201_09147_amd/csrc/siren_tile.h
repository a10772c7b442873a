// siren_tile.h -- fused SIREN evaluator for one wavefront tile on gfx950.
//
// Evaluates N(p) = W_K h_K + b_K, h_0 = p, h_{i+1} = sin(W_i h_i + b_i) (the MLP
// form of Eq.(2) with phi = sin) for the 32 columns of a wave tile:
//   * layer 0 (d_in -> H) as 32x32x2 fp32 MFMAs over the augmented input
//     (x, y, z[, t], 1): the bias rides in the A operand, the argument stays
//     float32 (omega0 = 30 makes it large);
//   * hidden layers (H -> H) as 32x32 MFMA GEMMs in the stack's precision:
//     A = packed weights streamed from L2 (one 16-byte load per lane per
//     32x32x16 bf16/fp16 instruction, or per four 32x32x2 fp32 instructions),
//     B = the previous layer's activations held in registers, C = the bias;
//   * sin on the VALU (v_sin_f32 in revolutions), converted to the MFMA input
//     precision in registers;
//   * output layer as a per-lane dot product plus one cross-half reduction.
//
// Tangent mode (TAN) carries the analytic normal of Sec. 5.1 in the same pass:
// columns 4q+c hold [h | G_x G_y G_z] of point q.  Tangent column j enters
// layer 0 as the unit vector e_j with 0 in the bias slot, so its accumulator is
// W_0[:, j]; every layer then applies G_i = phi'(a_i) * (W_i G_{i-1}) -- the
// commuted Hadamard form of Alg. 2 whose i = 0 case is the initial condition
// G_0 = W_0[j] * phi'(a_0) -- with phi'(a_i) = cos taken from the primal column
// of the same quad (DPP broadcast).  The output layer gives grad N = W_K G.
// The forward is shared by the three tangent columns instead of being
// recomputed per coordinate.
#pragma once
#include <hip/hip_runtime.h>

#include "nnm_device.h"

namespace nnm {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr float kTwoPi = 6.28318530717958647692f;

// Depth (in k-steps) of the register ring that prefetches hidden-layer A
// fragments from L2.
#ifndef NNM_RING_FP32
#define NNM_RING_FP32 2
#endif
#ifndef NNM_RING_LOWP
#define NNM_RING_LOWP 4
#endif
// Ring depth for H = 64 (its four k-steps fit a depth-4 ring; a shallower ring
// frees registers for occupancy).
#ifndef NNM_RING_LOWP_64
#define NNM_RING_LOWP_64 4
#endif

// Compiler barrier: memory operations are not moved across it, which keeps
// loop-invariant table reads from being hoisted into long-lived registers.
#define NNM_MEM_FENCE() __asm__ volatile("" ::: "memory")

// Widths whose first-layer operand and first hidden layer are held in LDS
// (then the tile's only global loads are its rays': a prefetch of ray data is
// not caught by waits on weight loads, and the weights come at LDS latency).
#ifndef NNM_LDS_WEIGHTS_MAX_H
#define NNM_LDS_WEIGHTS_MAX_H 64
#endif

// Per-workgroup copy of the per-network tables (read with broadcast) and, for
// narrow networks, of the first two layers' MFMA operands.
template <int H>
struct NetSmem {
  static constexpr bool kCache = H <= NNM_LDS_WEIGHTS_MAX_H;
  float wk[H];                   // output weights, accumulator layout
  float bh[(kMaxSine - 1) * H];  // hidden biases / 2 pi, accumulator layout
  float a0[kCache ? 3 * (H / 32) * 64 : 1];  // layer-0 A operand (copy of DevLevel::a0)
  uint4 ah1[kCache ? H * H / 4 : 1];         // hidden layer 1 A fragments (H * H * 4 bytes: the fp32 size)
};

template <int H>
__device__ inline void stage_net(NetSmem<H>* sm, const DevLevel& L) {
  for (int i = threadIdx.x; i < H; i += blockDim.x) sm->wk[i] = L.wk[i];
  const int nb = (L.n_sine - 1) * H;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) sm->bh[i] = L.bh[i];
  if constexpr (NetSmem<H>::kCache) {
    for (int i = threadIdx.x; i < 3 * (H / 32) * 64; i += blockDim.x) sm->a0[i] = L.a0[i];
    if (L.n_sine >= 2) {
      // one hidden layer: ah_stride bytes (H * H * element size, at most the array)
      const int n16 = (int)min((long long)(H * H / 4), L.ah_stride / 16);
      const uint4* src = (const uint4*)L.ah;
      for (int i = threadIdx.x; i < n16; i += blockDim.x) sm->ah1[i] = src[i];
    }
  }
  __syncthreads();
}

__device__ inline float sin_rev(float r) { return __builtin_amdgcn_sinf(r); }
__device__ inline float cos_rev(float r) { return __builtin_amdgcn_cosf(r); }
__device__ inline float fract_rev(float r) { return __builtin_amdgcn_fractf(r); }

// v of lane l plus v of lane l ^ 32, the same sum (lower half first) on both
// halves: one v_permlane32_swap exchanges the halves.
__device__ inline float half_sum(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Value of lane 4*(l/4)+SEL broadcast to the four lanes of each quad.
template <int SEL>
__device__ inline float quad_bcast(float v) {
  constexpr int ctrl = SEL | (SEL << 2) | (SEL << 4) | (SEL << 6);  // quad_perm [SEL x4]
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, 0xF, 0xF, false));
}

template <int P>
struct HiddenOps;

template <>
struct HiddenOps<PREC_BF16> {
  typedef bf16x8_t frag_t;
  static __device__ inline frag_t pack(const float* v) {
    frag_t f;
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = (__bf16)v[e];
    return f;
  }
  static __device__ inline f32x16_t mfma(frag_t a, frag_t b, f32x16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

template <>
struct HiddenOps<PREC_FP16> {
  typedef f16x8_t frag_t;
  static __device__ inline frag_t pack(const float* v) {
    frag_t f;
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = (_Float16)v[e];
    return f;
  }
  static __device__ inline f32x16_t mfma(frag_t a, frag_t b, f32x16_t c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

// Layer-0 B operand of k-step ks for lane half g: element 2 ks + g of the
// augmented input (x, y, z, 1) or (x, y, z, t, 1, 0); tangent columns use the
// unit vector of their coordinate with 0 in the bias and time slots.
__device__ inline float layer0_input(float4 in, int d_in, int c, int ks, int g) {
  const int k = 2 * ks + g;
  if (c > 0) return (k == c - 1) ? 1.f : 0.f;
  if (k < 3) return k == 0 ? in.x : (k == 1 ? in.y : in.z);
  if (d_in == 4) return k == 3 ? in.w : (k == 4 ? 1.f : 0.f);
  return k == 3 ? 1.f : 0.f;
}

// Inf-norm of a network input (x, y, z[, t]).
__device__ inline float input_norm(float4 in, int d_in) {
  return fmaxf(fmaxf(fabsf(in.x), fabsf(in.y)), fmaxf(fabsf(in.z), d_in == 4 ? fabsf(in.w) : 0.f));
}

// acc += A b over an H x H layer with 32x32x2 fp32 MFMAs: k-step ks uses
// b[ks/16][ks%16] (accumulator layout of the previous layer); A packed as
// f32x4 groups of four k-steps, streamed through a register ring.
template <int H>
__device__ inline void gemm_fp32(const float (&b)[H / 32][16], const f32x4_t* A, f32x16_t* acc) {
  constexpr int MB = H / 32;
  constexpr int NQ = H / 8;
  constexpr int kRing = NNM_RING_FP32;
  const int lane = threadIdx.x & 63;
  f32x4_t ring[kRing][MB];
#pragma unroll
  for (int d = 0; d < kRing; ++d)
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) ring[d][mb] = A[(d * MB + mb) * 64 + lane];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int ks = 4 * q + e;
      const float bv = b[ks / 16][ks % 16];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
        acc[mb] = __builtin_amdgcn_mfma_f32_32x32x2f32(ring[q % kRing][mb][e], bv, acc[mb], 0, 0, 0);
    }
    if (q + kRing < NQ) {
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) ring[q % kRing][mb] = A[((q + kRing) * MB + mb) * 64 + lane];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int H, int P, bool TAN>
struct SirenTile {
  static constexpr int MB = H / 32;
  float act[MB][16];  // activations of the current layer, accumulator layout

  // h = sin(a) for primal columns; G = 2 pi v cos(a) for tangent columns, a the
  // primal accumulator of the same quad.  Accumulators are in revolutions
  // (weights / 2 pi); tangent accumulators carry (W / 2 pi) G, hence the 2 pi.
  //
  // One sine per element: cos(2 pi r) = sin(2 pi (r + 1/4)), so tangent lanes
  // shift the argument by a quarter revolution and scale by 2 pi v.  RED adds
  // the reduction to [0, 1) revolutions (first layer, or wide argument bounds).
  template <bool RED>
  __device__ inline void activate_r(const f32x16_t* acc, int c) {
    const float off = c ? 0.25f : 0.f, m1 = c ? kTwoPi : 0.f, m0 = c ? 0.f : 1.f;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float v = acc[mb][r];
        if (TAN) {
          float rp = quad_bcast<0>(v) + off;
          if (RED) rp = fract_rev(rp);
          act[mb][r] = sin_rev(rp) * fmaf(v, m1, m0);
        } else {
          act[mb][r] = sin_rev(RED ? fract_rev(v) : v);
        }
      }
  }

  // reduce is uniform (per level): a branch, not a per-element select
  __device__ inline void activate(const f32x16_t* acc, int c, bool reduce) {
    if (reduce)
      activate_r<true>(acc, c);
    else
      activate_r<false>(acc, c);
  }

  // Layer-0 accumulators: W_0 [in | 1] / 2 pi (tangent columns: W_0[:, c-1] / 2 pi).
  __device__ inline void layer0_acc(const NetSmem<H>* sm, const DevLevel& L, float4 in, int c, f32x16_t* acc) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 5;
    const int ks0 = L.d_in == 4 ? 3 : 2;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mb][r] = 0.f;
    const float* A = NetSmem<H>::kCache ? sm->a0 : L.a0;
#pragma unroll
    for (int ks = 0; ks < 3; ++ks) {
      if (ks < ks0) {
        const float b = layer0_input(in, L.d_in, c, ks, g);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
          acc[mb] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[(ks * MB + mb) * 64 + lane], b, acc[mb], 0, 0, 0);
      }
    }
  }

  // The first layer's sine arguments need the reduction to [0, 1) revolutions
  // unless every column's input is within L.l0_safe (inf-norm), the bound
  // below which they stay within 63 revolutions (checked per wave).
  __device__ inline void first_layer(const NetSmem<H>* sm, const DevLevel& L, float4 in, int c) {
    f32x16_t acc[MB];
    layer0_acc(sm, L, in, c, acc);
    activate(acc, c, !__all(input_norm(in, L.d_in) <= L.l0_safe));
  }

  // Hidden-layer accumulators W_i act / 2 pi + b_i / 2 pi (bias on primal columns).
  __device__ inline void hidden_acc(const NetSmem<H>* sm, const DevLevel& L, int layer, int c, f32x16_t* acc) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 5;
    NNM_MEM_FENCE();
    const float* bias = sm->bh + (layer - 1) * H;
    // C = bias for primal columns; tangent columns carry W G only.
    const bool primal = !TAN || c == 0;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mb][r] = primal ? bias[acc_slot(mb, g, r)] : 0.f;
    if (NetSmem<H>::kCache && layer == 1)
      hidden_gemm((const char*)sm->ah1, acc);  // LDS
    else
      hidden_gemm((const char*)L.ah + (long long)(layer - 1) * L.ah_stride, acc);
  }

  // acc += A act for one hidden layer, A read from `base` (global memory or LDS).
  __device__ inline void hidden_gemm(const char* base, f32x16_t* acc) {
    const int lane = threadIdx.x & 63;
    if constexpr (P == PREC_FP32) {
      gemm_fp32<H>(act, (const f32x4_t*)base, acc);
    } else {
      typedef HiddenOps<P> Ops;
      typedef typename Ops::frag_t frag_t;
      constexpr int KS = 2 * MB;
      // never deeper than the layer's k-steps (no fragment past the layer is read)
      constexpr int kRingWant = H == 64 ? NNM_RING_LOWP_64 : NNM_RING_LOWP;
      constexpr int kRing = kRingWant < KS ? kRingWant : KS;
      frag_t bfr[KS];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        bfr[2 * mb] = Ops::pack(&act[mb][0]);
        bfr[2 * mb + 1] = Ops::pack(&act[mb][8]);
      }
      const frag_t* A = (const frag_t*)base;
      frag_t ring[kRing][MB];
#pragma unroll
      for (int d = 0; d < kRing; ++d)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) ring[d][mb] = A[(d * MB + mb) * 64 + lane];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[mb] = Ops::mfma(ring[ks % kRing][mb], bfr[ks], acc[mb]);
        if (ks + kRing < KS) {
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) ring[ks % kRing][mb] = A[((ks + kRing) * MB + mb) * 64 + lane];
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }

  __device__ inline void hidden_layer(const NetSmem<H>* sm, const DevLevel& L, int layer, int c) {
    f32x16_t acc[MB];
    hidden_acc(sm, L, layer, c, acc);
    activate(acc, c, L.reduce_hidden != 0);
  }

  // Output layer, this lane's half: the dot of W_K with the 16 MB rows the
  // lane holds (the column's other rows sit in lane l ^ 32).
  __device__ inline float output_part(const NetSmem<H>* sm) {
    const int g = (threadIdx.x & 63) >> 5;
    NNM_MEM_FENCE();
    float part = 0.f;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) part = fmaf(sm->wk[acc_slot(mb, g, r)], act[mb][r], part);
      __builtin_amdgcn_sched_barrier(0);
    }
    return part;
  }

  // Output layer on the current activations: per lane, the reduced value of
  // its column (N for primal columns, dN/dx_{c-1} for tangent columns).
  __device__ inline float output(const NetSmem<H>* sm, const DevLevel& L, int c) {
    float part = half_sum(output_part(sm));
    if (!TAN || c == 0) part += L.bk_dev ? *L.bk_dev : L.bk;
    return part;
  }

  // Returns, per lane, the output of its column after the cross-half reduction:
  // forward mode N (same on both halves); tangent mode N for c == 0 and
  // dN/dx_{c-1} for c = 1..3.
  __device__ inline float eval(const NetSmem<H>* sm, const DevLevel& L, float4 in, int c) {
    NNM_MEM_FENCE();
    first_layer(sm, L, in, c);
    for (int layer = 1; layer < L.n_sine; ++layer) hidden_layer(sm, L, layer, c);
    return output(sm, L, c);
  }
};

// Two forward tiles of one wave evaluated layer by layer side by side, so the
// MFMAs of one overlap the other's sines: tile 0's column n is the point in0
// of lane n, tile 1's column n the point in1 of lane n (both inputs the same
// on the two halves).  Returns, per lane l, N of column l % 32 of tile l / 32:
// with in0 / in1 taken from lanes n / n + 32, every lane gets the value at its
// own point.  Each column's value is computed as by SirenTile::eval (same
// operations, same order), apart from the first layer's reduction, which here
// is decided over both tiles.
template <int H, int P>
struct SirenPair {
  static constexpr int MB = H / 32;
  SirenTile<H, P, false> t0, t1;

  __device__ inline void activate(const f32x16_t* a0, const f32x16_t* a1, bool reduce) {
    if (reduce) {
      t0.template activate_r<true>(a0, 0);
      t1.template activate_r<true>(a1, 0);
    } else {
      t0.template activate_r<false>(a0, 0);
      t1.template activate_r<false>(a1, 0);
    }
  }

  __device__ inline float eval(const NetSmem<H>* sm, const DevLevel& L, float4 in0, float4 in1) {
    NNM_MEM_FENCE();
    f32x16_t a0[MB], a1[MB];
    t0.layer0_acc(sm, L, in0, 0, a0);
    t1.layer0_acc(sm, L, in1, 0, a1);
    activate(a0, a1, !__all(fmaxf(input_norm(in0, L.d_in), input_norm(in1, L.d_in)) <= L.l0_safe));
    for (int layer = 1; layer < L.n_sine; ++layer) {
      t0.hidden_acc(sm, L, layer, 0, a0);
      t1.hidden_acc(sm, L, layer, 0, a1);
      activate(a0, a1, L.reduce_hidden != 0);
    }
    // One v_permlane32_swap pairs the halves: the first result holds tile 0's
    // lower-half partials then tile 1's, the second the upper halves'.
    const float p0 = t0.output_part(sm), p1 = t1.output_part(sm);
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(p0), __float_as_uint(p1), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]) + (L.bk_dev ? *L.bk_dev : L.bk);
  }
};

// Value of lane l % 32 (LO) or of lane 32 + l % 32 (!LO) on every lane.
template <bool LO>
__device__ inline float half_bcast(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return __uint_as_float(LO ? r[0] : r[1]);
}
template <bool LO>
__device__ inline float4 half_bcast4(float4 v) {
  return make_float4(half_bcast<LO>(v.x), half_bcast<LO>(v.y), half_bcast<LO>(v.z), half_bcast<LO>(v.w));
}

}  // namespace nnm

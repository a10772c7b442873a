// trace_ws.hip -- weight-stationary tracing and normal kernels for width-256
// networks with two hidden layers in bf16 / fp16 (the fine level of the
// nested stacks).
//
// A workgroup is four waves, one per SIMD.  Wave w keeps rows [64 w, 64 w + 64)
// of both hidden weight matrices in registers for the whole kernel (2 x 32 KB
// per wave), so the hidden weights are read from memory once per workgroup
// instead of once per tile.  A tile is 64 columns (64 rays, or 16 points x
// [h | G_x G_y G_z] in the normal pass).  Each layer:
//   * every wave multiplies its 64 rows by all 256 inputs of the 64 columns
//     (32x32x16 MFMAs: A = its stationary weights, B = the previous layer's
//     activations read from LDS, C = the bias);
//   * applies sin (revolutions) to its rows and writes them, as 16-bit values,
//     into the LDS activation buffer of the next layer;
//   * a barrier publishes the rows to the other waves.
// Layer 0 is a 32x32x2 fp32 MFMA over (x, y, z[, t], 1) per wave; the last
// layer's activations stay in float32 and feed the output dot product as
// per-wave partial sums combined through LDS.  Wave 0 runs the sphere-tracing
// control (slot refill from the segmented queue, the Algorithm 1 update,
// compaction into the next queue) on 64 slots, one per lane.
#include "trace_common.h"

namespace nnm {

constexpr int kWsCols = 64;         // columns per workgroup tile
constexpr int kWsStride = 256 + 8;  // 16-bit elements per LDS column (padding spreads LDS banks)

struct WsSmem {
  uint16_t act[2][kWsCols * kWsStride];
  float bias[2][256];
  float wk[256];
  float part[4][kWsCols];
  float4 xin[kWsCols];
  int flag;
  int ring[2 * kPushBatch];
};

template <int P>
struct WsBits;
template <>
struct WsBits<PREC_BF16> {
  static __device__ inline uint16_t bits(float v) {
    const __bf16 h = (__bf16)v;
    return __builtin_bit_cast(uint16_t, h);
  }
};
template <>
struct WsBits<PREC_FP16> {
  static __device__ inline uint16_t bits(float v) {
    const _Float16 h = (_Float16)v;
    return __builtin_bit_cast(uint16_t, h);
  }
};

// Stationary state of one wave: its rows of the layer-0 A operand and of both
// hidden weight matrices.
template <int P>
struct WsWeights {
  typedef typename HiddenOps<P>::frag_t frag_t;
  float w0[2][3];
  frag_t w1[2][16];
  frag_t w2[2][16];

  __device__ inline void load(const DevLevel& L, int wave, int lane) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int ks = 0; ks < 3; ++ks) w0[rb][ks] = L.ws_a0[((wave * 2 + rb) * 3 + ks) * 64 + lane];
    const frag_t* WA = (const frag_t*)L.ws_ah;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) {
        w1[rb][ks] = WA[(((0 * 4 + wave) * 2 + rb) * 16 + ks) * 64 + lane];
        w2[rb][ks] = WA[(((1 * 4 + wave) * 2 + rb) * 16 + ks) * 64 + lane];
      }
  }
};

__device__ inline int ws_row(int wave, int rb, int g, int r) { return 64 * wave + 32 * rb + 8 * (r / 4) + 4 * g + (r % 4); }

// One wave's part of a tile evaluation.  TAN: columns 4q+c are [h | G].
// Returns, per lane and column block, this wave's partial output sum.
template <int P, bool TAN>
__device__ inline void ws_eval(WsSmem& sm, const WsWeights<P>& W, const DevLevel& L, float part[2]) {
  typedef HiddenOps<P> Ops;
  typedef typename Ops::frag_t frag_t;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, j = lane & 31, g = lane >> 5;
  const int c = j & 3;  // column role in the tangent mode
  const int ks0 = L.d_in == 4 ? 3 : 2;
  f32x16_t acc[2][2];
  // ---- layer 0 (fp32 MFMA over the augmented input)
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const float4 in = sm.xin[32 * cb + j];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[cb][rb][r] = 0.f;
#pragma unroll
      for (int ks = 0; ks < 3; ++ks)
        if (ks < ks0)
          acc[cb][rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(W.w0[rb][ks], layer0_input(in, L.d_in, TAN ? c : 0, ks, g),
                                                             acc[cb][rb], 0, 0, 0);
    }
  }
  // ---- three activations: layer 0 -> act[0], hidden 1 -> act[1], hidden 2 -> output
#pragma unroll
  for (int stage = 0; stage < 3; ++stage) {
    if (stage > 0) {
      const uint16_t* src = sm.act[stage - 1];
      const float* bias = sm.bias[stage - 1];
      const bool primal = !TAN || c == 0;
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[cb][rb][r] = primal ? bias[ws_row(wave, rb, g, r)] : 0.f;
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) {
        frag_t b[2];
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) b[cb] = *(const frag_t*)&src[(32 * cb + j) * kWsStride + 16 * ks + 8 * g];
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
          for (int rb = 0; rb < 2; ++rb)
            acc[cb][rb] = Ops::mfma(stage == 1 ? W.w1[rb][ks] : W.w2[rb][ks], b[cb], acc[cb][rb]);
      }
    }
    const bool reduce = stage == 0 || L.reduce_hidden;
    if (stage < 2) {
      uint16_t* dst = sm.act[stage];
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int b4 = 0; b4 < 4; ++b4) {
            uint16_t h[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const float v = acc[cb][rb][4 * b4 + i];
              float a;
              if (TAN) {
                // one sine per lane: sin(2 pi r) on primal columns, cos(2 pi r) =
                // sin(2 pi (r + 1/4)) on tangent columns (r reduced to [0, 1) first)
                const float rp = fract_rev(quad_bcast<0>(v));
                const float sv = sin_rev(c == 0 ? rp : rp + 0.25f);
                a = (c == 0) ? sv : (kTwoPi * v) * sv;
              } else {
                a = sin_rev(reduce ? fract_rev(v) : v);
              }
              h[i] = WsBits<P>::bits(a);
            }
            const int row = 64 * wave + 32 * rb + 8 * b4 + 4 * g;
            uint2 packed;
            packed.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
            packed.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
            *(uint2*)&dst[(32 * cb + j) * kWsStride + row] = packed;
          }
      __syncthreads();
    } else {
      // last hidden layer: float32 activations into the output dot product
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        float s = 0.f;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const float v = acc[cb][rb][r];
            float a;
            if (TAN) {
              const float rp = fract_rev(quad_bcast<0>(v));
              const float sv = sin_rev(c == 0 ? rp : rp + 0.25f);
              a = (c == 0) ? sv : (kTwoPi * v) * sv;
            } else {
              a = sin_rev(reduce ? fract_rev(v) : v);
            }
            s = fmaf(sm.wk[ws_row(wave, rb, g, r)], a, s);
          }
        part[cb] = s + __shfl_xor(s, 32);
      }
    }
  }
}

template <int P>
__global__ void __launch_bounds__(kBlockThreads, 1) k_trace_ws(TraceLevelArgs A) {
  __shared__ WsSmem sm;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = (lane >> 5);
  const DevLevel& L = A.L;
  WsWeights<P> W;
  W.load(L, wave, lane);
  for (int i = threadIdx.x; i < 256; i += blockDim.x) {
    sm.bias[0][i] = L.bh_plain[i];
    sm.bias[1][i] = L.bh_plain[256 + i];
    sm.wk[i] = L.wk_plain[i];
  }
  __syncthreads();
  // Wave 0: one slot per lane; a 64-entry staging ring of prefetched rays
  // (lane e holds ring entry e) refills empty slots through lane shuffles, and
  // is topped up right after, so its loads complete during the evaluation.
  const int n_in = A.in_count ? *A.in_count : A.n;
  int ray = -1, k = 0, st = 0;
  float tau = 0.f, ox = 0.f, oy = 0.f, oz = 0.f, vx = 0.f, vy = 0.f, vz = 0.f, tt = 0.f, x = 0.f, y = 0.f, z = 0.f,
        cx = 0.f, cy = 0.f;
  int s_ray = -1, s_st = 0;
  float s_ox = 0.f, s_oy = 0.f, s_oz = 0.f, s_vx = 0.f, s_vy = 0.f, s_vz = 0.f, s_tt = 0.f, s_tau = 0.f;
  int s_head = 0, s_count = 0;
  int cur = 0, end = 0, ring_start = 0, ring_n = 0;
  const int chunk = min(kChunk, max(64, (n_in / (8 * (int)gridDim.x)) & ~63));
  const int seg_len = (n_in + kSegments - 1) / kSegments;
  int seg = blockIdx.x % kSegments, seg_tries = 0;
  bool exhausted = false;
  for (;;) {
    if (wave == 0) {
      bool live;
      for (;;) {
        // consume staged rays into empty slots
        const unsigned long long emask = __ballot(ray < 0);
        const int take = min(__popcll(emask), s_count);
        const int p = __popcll(emask & ((1ull << lane) - 1ull));
        const bool fill = ray < 0 && p < take;
        const int src = fill ? ((s_head + p) & 63) : lane;
        const int n_ray = __shfl(s_ray, src), n_st = __shfl(s_st, src);
        const float n_ox = __shfl(s_ox, src), n_oy = __shfl(s_oy, src), n_oz = __shfl(s_oz, src);
        const float n_vx = __shfl(s_vx, src), n_vy = __shfl(s_vy, src), n_vz = __shfl(s_vz, src);
        const float n_tt = __shfl(s_tt, src), n_tau = __shfl(s_tau, src);
        if (fill) {
          ray = n_ray;
          st = n_st;
          ox = n_ox;
          oy = n_oy;
          oz = n_oz;
          vx = n_vx;
          vy = n_vy;
          vz = n_vz;
          tt = n_tt;
          tau = n_tau;
          k = 0;
        }
        s_head = (s_head + take) & 63;
        s_count -= take;
        // top the staging ring up with new queue entries (loads issued, not awaited)
        while (s_count < 64 && !exhausted) {
          if (cur >= end) {
            const int s0 = seg * seg_len;
            const int s_len = max(0, min(seg_len, n_in - s0));
            int base = 0;
            if (lane == 0) base = atomicAdd(A.in_heads + seg * kHeadStride, chunk);
            base = __shfl(base, 0);
            if (base >= s_len) {
              seg = (seg + 1) % kSegments;
              if (++seg_tries >= kSegments) exhausted = true;
              continue;
            }
            cur = s0 + base;
            end = s0 + min(base + chunk, s_len);
          }
          const int add = min(64 - s_count, end - cur);
          const int q = ((lane - s_head) & 63) - s_count;
          if (q >= 0 && q < add) {
            const int idx = cur + q;
            s_ray = A.in_queue ? A.in_queue[idx] : idx;
            s_ox = A.o[3 * s_ray + 0];
            s_oy = A.o[3 * s_ray + 1];
            s_oz = A.o[3 * s_ray + 2];
            s_vx = A.v[3 * s_ray + 0];
            s_vy = A.v[3 * s_ray + 1];
            s_vz = A.v[3 * s_ray + 2];
            s_tt = A.t ? A.t[s_ray] : 0.f;
            if (A.level == 0) {
              s_tau = 0.f;
              s_st = 0;
              if (A.steps)
                for (int jj = 1; jj < A.m; ++jj) A.steps[(long long)s_ray * A.m + jj] = 0;
            } else {
              s_tau = A.depth[s_ray];
              s_st = A.status[s_ray];
            }
          }
          s_count += add;
          cur += add;
        }
        live = __ballot(ray >= 0) != 0ull;
        // an empty tile while rays are still staged: consume again
        if (live || s_count == 0) break;
      }
      x = fmaf(tau, vx, ox);
      y = fmaf(tau, vy, oy);
      z = fmaf(tau, vz, oz);
      center_at(A.B, tt, cx, cy);
      sm.xin[lane] = net_input(L, x, y, z, tt, cx, cy);
      if (lane == 0) sm.flag = live ? 1 : 0;
    }
    __syncthreads();
    if (sm.flag == 0) break;
    float part[2];
    ws_eval<P, false>(sm, W, L, part);
    if (g == 0) {
      sm.part[wave][lane] = part[0];
      sm.part[wave][32 + lane] = part[1];
    }
    __syncthreads();
    if (wave == 0) {
      const float N = sm.part[0][lane] + sm.part[1][lane] + sm.part[2][lane] + sm.part[3][lane] + L.bk;
      int outcome = 0;
      if (ray >= 0) {
        float base_term = 0.f;
        if (A.B.sphere) {
          const float dx = x - cx, dy = y - cy;
          base_term = sqrtf(fmaf(dx, dx, fmaf(dy, dy, z * z))) - A.B.r0;
        }
        const float f = fmaf(L.amplitude, N, base_term);
        const float d = f - A.delta;
        ++k;
        if (!isfinite(d)) {
          st |= ST_NONFINITE;
          outcome = 2;
        } else {
          if (d < 0.f) st |= ST_NEG_STEP;
          tau = fmaf(A.step_scale, d, tau);
          if (tau > A.far) {
            st |= ST_FAR;
            outcome = 2;
          } else if (d <= A.eps) {
            outcome = 1;
          } else if (k >= A.max_steps) {
            st |= ST_BUDGET;
            outcome = 2;
          }
        }
      }
      const unsigned long long pmask = __ballot(outcome == 1);
      if (pmask && A.out_queue) {
        if (outcome == 1) sm.ring[(ring_start + ring_n + __popcll(pmask & ((1ull << lane) - 1ull))) & (2 * kPushBatch - 1)] = ray;
        ring_n += __popcll(pmask);
        if (ring_n >= kPushBatch) {
          __builtin_amdgcn_wave_barrier();
          int base = 0;
          if (lane == 0) base = atomicAdd(A.out_count, kPushBatch);
          base = __shfl(base, 0);
          A.out_queue[base + lane] = sm.ring[(ring_start + lane) & (2 * kPushBatch - 1)];
          __builtin_amdgcn_wave_barrier();
          ring_start = (ring_start + kPushBatch) & (2 * kPushBatch - 1);
          ring_n -= kPushBatch;
        }
      }
      if (outcome != 0) {
        if (A.steps) A.steps[(long long)ray * A.m + A.level] = (uint8_t)k;
        if (outcome == 2) {
          A.depth[ray] = __builtin_inff();
          A.hit[ray] = 0;
          A.status[ray] = (uint8_t)st;
          if (A.normal) {
            A.normal[3 * ray + 0] = 0.f;
            A.normal[3 * ray + 1] = 0.f;
            A.normal[3 * ray + 2] = 0.f;
          }
        } else if (A.is_final) {
          A.depth[ray] = tau;
          A.hit[ray] = 1;
          A.status[ray] = (uint8_t)(st | ST_HIT);
        } else {
          A.depth[ray] = tau;
          A.status[ray] = (uint8_t)st;
        }
        ray = -1;
      }
    }
  }
  if (wave == 0 && ring_n > 0 && A.out_queue) {
    __builtin_amdgcn_wave_barrier();
    int base = 0;
    if (lane == 0) base = atomicAdd(A.out_count, ring_n);
    base = __shfl(base, 0);
    if (lane < ring_n) A.out_queue[base + lane] = sm.ring[(ring_start + lane) & (2 * kPushBatch - 1)];
  }
}

template <int P>
__global__ void __launch_bounds__(kBlockThreads, 1) k_normal_ws(NormalArgs A) {
  __shared__ WsSmem sm;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 5;
  const DevLevel& L = A.L;
  WsWeights<P> W;
  W.load(L, wave, lane);
  for (int i = threadIdx.x; i < 256; i += blockDim.x) {
    sm.bias[0][i] = L.bh_plain[i];
    sm.bias[1][i] = L.bh_plain[256 + i];
    sm.wk[i] = L.wk_plain[i];
  }
  __syncthreads();
  const int n_in = A.count ? *A.count : A.n;
  const int q = lane >> 2, c = lane & 3;  // wave 0: lane = column, 16 points x 4 columns
  for (int base = blockIdx.x * 16; base < n_in; base += gridDim.x * 16) {
    int ray = -1;
    float x = 0.f, y = 0.f, z = 0.f, tt = 0.f, cx = 0.f, cy = 0.f;
    if (wave == 0) {
      const int slot = base + q;
      ray = (slot < n_in) ? (A.queue ? A.queue[slot] : slot) : -1;
      if (ray >= 0) {
        const float tau = A.depth[ray];
        x = fmaf(tau, A.v[3 * ray + 0], A.o[3 * ray + 0]);
        y = fmaf(tau, A.v[3 * ray + 1], A.o[3 * ray + 1]);
        z = fmaf(tau, A.v[3 * ray + 2], A.o[3 * ray + 2]);
        tt = A.t ? A.t[ray] : 0.f;
      }
      center_at(A.B, tt, cx, cy);
      sm.xin[lane] = net_input(L, x, y, z, tt, cx, cy);
    }
    __syncthreads();
    float part[2];
    ws_eval<P, true>(sm, W, L, part);
    if (g == 0) {
      sm.part[wave][lane] = part[0];
      sm.part[wave][32 + lane] = part[1];
    }
    __syncthreads();
    if (wave == 0) {
      float val = sm.part[0][lane] + sm.part[1][lane] + sm.part[2][lane] + sm.part[3][lane];
      if (c == 0) val += L.bk;
      const float gx = quad_bcast<1>(val), gy = quad_bcast<2>(val), gz = quad_bcast<3>(val);
      if (c == 0 && ray >= 0) {
        float fx = L.amplitude * gx, fy = L.amplitude * gy, fz = L.amplitude * gz;
        if (A.B.sphere) {
          const float dx = x - cx, dy = y - cy;
          const float r = sqrtf(fmaf(dx, dx, fmaf(dy, dy, z * z)));
          if (r > 0.f) {
            fx += dx / r;
            fy += dy / r;
            fz += z / r;
          }
        }
        const float len = sqrtf(fmaf(fx, fx, fmaf(fy, fy, fz * fz)));
        const float inv = len > 0.f ? 1.f / len : 0.f;
        A.normal[3 * ray + 0] = fx * inv;
        A.normal[3 * ray + 1] = fy * inv;
        A.normal[3 * ray + 2] = fz * inv;
      }
    }
  }
}

hipError_t launch_trace_ws(int prec, const TraceLevelArgs& a, int grid, hipStream_t s) {
  if (prec == PREC_BF16)
    hipLaunchKernelGGL(k_trace_ws<PREC_BF16>, dim3(grid), dim3(kBlockThreads), 0, s, a);
  else if (prec == PREC_FP16)
    hipLaunchKernelGGL(k_trace_ws<PREC_FP16>, dim3(grid), dim3(kBlockThreads), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_normal_ws(int prec, const NormalArgs& a, int grid, hipStream_t s) {
  if (prec == PREC_BF16)
    hipLaunchKernelGGL(k_normal_ws<PREC_BF16>, dim3(grid), dim3(kBlockThreads), 0, s, a);
  else if (prec == PREC_FP16)
    hipLaunchKernelGGL(k_normal_ws<PREC_FP16>, dim3(grid), dim3(kBlockThreads), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

int ws_resident_blocks(int prec, int kind, int device) {
  const void* fn = prec == PREC_FP16 ? (kind == 0 ? (const void*)k_trace_ws<PREC_FP16> : (const void*)k_normal_ws<PREC_FP16>)
                                     : (kind == 0 ? (const void*)k_trace_ws<PREC_BF16> : (const void*)k_normal_ws<PREC_BF16>);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlockThreads, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
  return per_cu * cus;
}

}  // namespace nnm

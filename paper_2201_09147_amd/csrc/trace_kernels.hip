// trace_kernels.hip -- multiscale sphere tracing, analytic normals and point
// evaluation kernels for gfx950.
//
// Multiscale sphere tracing (Algorithm 1 of the paper) runs one persistent
// kernel per level.  Each wavefront owns 32 ray slots (one tile column each,
// held by both lane halves) or, for narrow nets in bf16/fp16, 64 (one per
// lane, evaluated as two tiles side by side, which halves the per-ray control
// work) and loops: refill empty slots from the level's input queue (one
// atomic per chunk of entries), evaluate f_j at all slots with the fused
// SIREN tile, step every live ray (tau += s d with d = f_j - delta_j), and
// retire rays that left the level: to the next level's queue (d <= eps), to
// the hit queue (last level), or as a miss (tau > far, budget used,
// non-finite).  Slots freed by retired rays are refilled
// on the next iteration, so tiles stay dense while the queue lasts and every
// tile evaluates one network only.  The normal pass then evaluates the normal
// level's forward and three tangent columns (Sec. 5.1) at the hit points.
#include "trace_common.h"

namespace nnm {

__global__ void k_zero_ints(int* p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

// Waves per SIMD the tracing kernel of width H is compiled for (the register
// budget follows: 512 / waves per lane, VGPRs and accumulator registers together).
// Width 32 runs at its natural 5 (96 registers, no spills; at 6 waves, 80
// registers, it spills on the refill and push paths and runs 4% slower);
// width 64 gains nothing from 4 and loses at 5.
#ifndef NNM_TRACE_WAVES_32
#define NNM_TRACE_WAVES_32 5
#endif
#ifndef NNM_TRACE_WAVES_64
#define NNM_TRACE_WAVES_64 1
#endif
// Widths traced with one ray per lane (two tiles per wave; bf16 and fp16
// only: with fp32 hidden layers the matrix pipe sets the pace and the pairing
// gains nothing), and their waves per SIMD.
#ifndef NNM_TRACE_PAIR_MAX_H
#define NNM_TRACE_PAIR_MAX_H 64
#endif
#ifndef NNM_TRACE_PAIR_WAVES_32
#define NNM_TRACE_PAIR_WAVES_32 4
#endif
#ifndef NNM_TRACE_PAIR_WAVES_64
#define NNM_TRACE_PAIR_WAVES_64 2
#endif
constexpr bool trace_pair(int H, int P) { return P != PREC_FP32 && H <= NNM_TRACE_PAIR_MAX_H; }
template <int H, bool PAIR>
constexpr int trace_waves_per_eu() {
  return PAIR ? (H == 32 ? NNM_TRACE_PAIR_WAVES_32 : NNM_TRACE_PAIR_WAVES_64)
              : (H == 32 ? NNM_TRACE_WAVES_32 : (H == 64 ? NNM_TRACE_WAVES_64 : 1));
}

template <int H, int P, bool PAIR>
__global__ void __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(trace_waves_per_eu<H, PAIR>())))
k_trace_level(TraceLevelArgs A) {
  __shared__ NetSmem<H> sm;
  // Per-wave ring of rays that finished the level, flushed to the output queue
  // kPushBatch at a time (one atomic per batch, coalesced stores), and the
  // workgroup's count of pushed rays per order key.
  __shared__ int push_ring[kBlockThreads / 64][2 * kPushBatch];
  __shared__ uint8_t push_key[kBlockThreads / 64][2 * kPushBatch];
  __shared__ int key_hist[kOrderKeys];
  if (threadIdx.x < kOrderKeys) key_hist[threadIdx.x] = 0;
  stage_net<H>(&sm, A.L);  // (ends with a workgroup barrier)
  const int lane = threadIdx.x & 63;
  const int col = lane & 31;
  const int g = lane >> 5;
  // The lane's ray slot: its own (PAIR) or its tile column's, whose state
  // both halves hold and whose results the lower half writes.  Slot masks are
  // ballots restricted to one lane per slot.
  constexpr int kSlots = PAIR ? 64 : 32;
  const bool writer = PAIR || g == 0;
  const unsigned long long slot_lanes = PAIR ? ~0ull : 0xffffffffull;
  const unsigned long long below = (1ull << (PAIR ? lane : col)) - 1ull;
  int* ring = push_ring[threadIdx.x >> 6];
  uint8_t* ring_key = A.out_key ? push_key[threadIdx.x >> 6] : nullptr;
  const int n_in = A.in_count ? *A.in_count : A.n;
  SirenTile<H, P, false> tile;
  SirenPair<H, P> pair;
  int ray = -1, k = 0, st = 0;
  float tau = 0.f, ox = 0.f, oy = 0.f, oz = 0.f, vx = 0.f, vy = 0.f, vz = 0.f, tt = 0.f, cx = 0.f, cy = 0.f;
  // Wave-uniform work chunk [cur, end) of the input queue and push-ring state.
  // The queue is split into kSegments segments with one pop counter each
  // (separate cache lines, so the atomics spread over many addresses); a wave
  // starts in segment (wave id mod kSegments) and, when it is empty, moves on
  // to one that still holds entries (one read of all counters).
  // Chunks hold about n_in / (8 * resident waves) entries (kSlots..kChunk),
  // so every wave takes several chunks and the queue drains evenly.
  int cur = 0, end = 0;
  PushRing pr;
  const int nwaves = gridDim.x * (kBlockThreads / 64);
  const int wave_id = blockIdx.x * (kBlockThreads / 64) + (threadIdx.x >> 6);
  const int chunk = min(kChunk, max(kSlots, (n_in / (8 * nwaves)) & ~31));
  int seg = wave_id % kSegments;
  bool exhausted = false;
  for (;;) {
    // Refill empty slots from the wave's chunk, grabbing a new chunk of
    // queue entries (one atomic) when it runs dry.
    unsigned long long emask = __ballot(ray < 0) & slot_lanes;
    while (emask != 0u && !exhausted) {
      if (cur >= end) {
        int s0, s_len;
        segment_bounds(seg, n_in, s0, s_len);
        int base = 0;
        if (lane == 0) base = atomicAdd(A.in_heads + seg * kHeadStride, chunk);
        base = __shfl(base, 0);
        if (base >= s_len) {
          // this segment is drained: on to one that is not, if any
          seg = next_open_segment(A.in_heads, n_in, wave_id, lane);
          if (seg < 0) {
            exhausted = true;
            break;
          }
          continue;
        }
        cur = s0 + base;
        end = s0 + min(base + chunk, s_len);
      }
      const int avail = end - cur;
      const int cnt = __popcll(emask);
      const int take = min(cnt, avail);
      if (ray < 0) {
        const int pos = __popcll(emask & below);
        if (pos < take) {
          const int idx = cur + pos;
          ray = A.in_queue ? A.in_queue[idx] : idx;
          ox = A.o[3 * ray + 0];
          oy = A.o[3 * ray + 1];
          oz = A.o[3 * ray + 2];
          vx = A.v[3 * ray + 0];
          vy = A.v[3 * ray + 1];
          vz = A.v[3 * ray + 2];
          tt = A.t ? A.t[ray] : 0.f;
          center_at(A.B, tt, cx, cy);  // c(t) is fixed per ray: once, on entry
          k = 0;
          if (A.level == 0) {
            tau = 0.f;
            st = 0;
            if (A.steps && writer)
              for (int j = 1; j < A.m; ++j) A.steps[(long long)ray * A.m + j] = 0;
          } else {
            tau = A.depth[ray];
            st = A.status[ray];
          }
        }
      }
      cur += take;
      emask = __ballot(ray < 0) & slot_lanes;
    }
    if (__ballot(ray >= 0) == 0ull) break;

    const float x = fmaf(tau, vx, ox), y = fmaf(tau, vy, oy), z = fmaf(tau, vz, oz);
    const float4 in = net_input(A.L, x, y, z, tt, cx, cy);
    float N;
    if constexpr (PAIR) {
      // Tile 0 takes the rays of lanes 0..31, tile 1 those of lanes 32..63; a
      // half with no live ray is not evaluated.
      const unsigned long long lv = __ballot(ray >= 0);
      const float4 in0 = half_bcast4<true>(in), in1 = half_bcast4<false>(in);
      if ((unsigned int)lv != 0u && (lv >> 32) != 0ull)
        N = pair.eval(&sm, A.L, in0, in1);
      else
        N = tile.eval(&sm, A.L, (unsigned int)lv != 0u ? in0 : in1, 0);
    } else {
      N = tile.eval(&sm, A.L, in, 0);
    }

    int outcome = 0;  // 0: keep stepping, 1: left the level through d <= eps, 2: miss
    if (ray >= 0) {
      float base_term = 0.f;
      if (A.B.sphere) {
        const float dx = x - cx, dy = y - cy;
        base_term = base_radius(dx, dy, z) - A.B.r0;
      }
      const float f = fmaf(A.L.amplitude, N, base_term);
      outcome = alg1_step(A, f - A.delta, tau, k, st);
    }
    // Compaction: rays that finished the level enter the wave's push ring.
    if (A.out_queue) {
      const unsigned long long pm = __ballot(outcome == 1) & slot_lanes;
      if (pm) {
        pr.add(ring, ring_key, pm, outcome == 1 && writer, __popcll(pm & below), ray, order_key(k));
        if (pr.n >= kPushBatch) pr.publish(ring, ring_key, lane, A.out_count, A.out_queue, A.out_key, key_hist, false);
      }
    }
    if (outcome != 0) {
      if (writer) {
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
      }
      ray = -1;
    }
  }
  // Flush what is left in the push ring, then the workgroup's key counts.
  if (pr.n > 0 && A.out_queue) pr.publish(ring, ring_key, lane, A.out_count, A.out_queue, A.out_key, key_hist, true);
  if (A.out_key) {
    __syncthreads();
    if (threadIdx.x < kOrderKeys) {
      const int c = key_hist[threadIdx.x];
      if (c) atomicAdd(A.out_hist + threadIdx.x, c);
    }
  }
}

// Counting sort of a level's output queue by decreasing order key (the layout
// of QueueOrderArgs).  Workgroup b owns entries [b per, (b + 1) per) and takes
// them kOrderBatch at a time, held in registers: it counts their keys in LDS,
// reserves room in every key's run with one atomic per key, then scatters.
// The order inside a key's run is unspecified (results do not depend on the
// order rays are traced in).
constexpr int kOrderThreads = 1024;
constexpr int kOrderPerThread = 4;
constexpr int kOrderBatch = kOrderThreads * kOrderPerThread;
__global__ void __launch_bounds__(kOrderThreads) k_queue_order(QueueOrderArgs A) {
  __shared__ int cnt[kOrderKeys], first[kOrderKeys];
  const int t = threadIdx.x;
  // entries of all larger keys come first: a suffix sum over the key totals
  int larger = 0;
  if (t < kOrderKeys) {
    const int h = A.hist[t];
    int s = h;
    for (int d = 1; d < kOrderKeys; d <<= 1) {
      const int o = __shfl_down(s, d);
      if (t + d < kOrderKeys) s += o;
    }
    larger = s - h;
  }
  const int n = *A.count;
  const int per = (n + (int)gridDim.x - 1) / (int)gridDim.x;
  const int lo = blockIdx.x * per, hi = min(n, lo + per);
  for (int b0 = lo; b0 < hi; b0 += kOrderBatch) {  // (uniform over the workgroup)
    if (t < kOrderKeys) cnt[t] = 0;
    __syncthreads();
    int key[kOrderPerThread], ray[kOrderPerThread];
#pragma unroll
    for (int e = 0; e < kOrderPerThread; ++e) {
      const int i = b0 + t + e * kOrderThreads;
      key[e] = -1;
      if (i < hi) {
        key[e] = A.key[i];
        ray[e] = A.in[i];
      }
    }
#pragma unroll
    for (int e = 0; e < kOrderPerThread; ++e)
      if (key[e] >= 0) atomicAdd(&cnt[key[e]], 1);
    __syncthreads();
    if (t < kOrderKeys) {
      const int c = cnt[t];
      first[t] = larger + (c ? atomicAdd(A.fill + t, c) : 0);
      cnt[t] = 0;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kOrderPerThread; ++e) {
      if (key[e] < 0) continue;
      const int r = first[key[e]] + atomicAdd(&cnt[key[e]], 1);
      if (r < n) A.out[sorted_position(r, n)] = ray[e];
    }
    __syncthreads();  // cnt and first are rewritten by the next batch
  }
}

// Forward + three tangent columns at the hit points (or at given points); unit
// grad f as the normal.
template <int H, int P>
__global__ void __launch_bounds__(kBlockThreads) k_normal(NormalArgs A) {
  __shared__ NetSmem<H> sm;
  stage_net<H>(&sm, A.L);
  const int lane = threadIdx.x & 63;
  const int col = lane & 31;
  const int g = lane >> 5;
  const int q = col >> 2, c = col & 3;
  const int waves = kBlockThreads / 64;
  const int wave = blockIdx.x * waves + (threadIdx.x >> 6);
  const int nwaves = gridDim.x * waves;
  const int n_in = A.count ? *A.count : A.n;
  SirenTile<H, P, true> tile;
  for (int base = wave * 8; base < n_in; base += nwaves * 8) {
    const int slot = base + q;
    const int ray = (slot < n_in) ? (A.queue ? A.queue[slot] : slot) : -1;
    float x = 0.f, y = 0.f, z = 0.f, tt = 0.f;
    if (ray >= 0) {
      if (A.x) {
        x = A.x[3 * ray + 0];
        y = A.x[3 * ray + 1];
        z = A.x[3 * ray + 2];
      } else {
        const float tau = A.depth[ray];
        x = fmaf(tau, A.v[3 * ray + 0], A.o[3 * ray + 0]);
        y = fmaf(tau, A.v[3 * ray + 1], A.o[3 * ray + 1]);
        z = fmaf(tau, A.v[3 * ray + 2], A.o[3 * ray + 2]);
      }
      tt = A.t ? A.t[ray] : 0.f;
    }
    float cx, cy;
    center_at(A.B, tt, cx, cy);
    const float val = tile.eval(&sm, A.L, net_input(A.L, x, y, z, tt, cx, cy), c);
    const float gx = quad_bcast<1>(val), gy = quad_bcast<2>(val), gz = quad_bcast<3>(val);
    if (c == 0 && g == 0 && ray >= 0) {
      float fx = A.L.amplitude * gx, fy = A.L.amplitude * gy, fz = A.L.amplitude * gz;
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

// Value and raw gradient at points (analytic_normal / nnm_net_eval).
template <int H, int P>
__global__ void __launch_bounds__(kBlockThreads) k_points(PointsArgs A) {
  __shared__ NetSmem<H> sm;
  stage_net<H>(&sm, A.L);
  const int lane = threadIdx.x & 63;
  const int col = lane & 31;
  const int g = lane >> 5;
  const int q = col >> 2, c = col & 3;
  const int waves = kBlockThreads / 64;
  const int wave = blockIdx.x * waves + (threadIdx.x >> 6);
  const int nwaves = gridDim.x * waves;
  SirenTile<H, P, true> tile;
  for (int base = wave * 8; base < A.n; base += nwaves * 8) {
    const int i = base + q;
    const bool live = i < A.n;
    float x = 0.f, y = 0.f, z = 0.f, tt = 0.f;
    if (live) {
      const long long b = (long long)A.x_stride * i;
      x = A.x[b + 0];
      y = A.x[b + 1];
      z = A.x[b + 2];
      tt = A.x_stride == 4 ? A.x[b + 3] : (A.t ? A.t[i] : 0.f);
    }
    float cx, cy;
    center_at(A.B, tt, cx, cy);
    const float val = tile.eval(&sm, A.L, net_input(A.L, x, y, z, tt, cx, cy), c);
    const float gx = quad_bcast<1>(val), gy = quad_bcast<2>(val), gz = quad_bcast<3>(val);
    if (c == 0 && g == 0 && live) {
      if (A.raw) {
        if (A.value) A.value[i] = val;
        if (A.grad) {
          A.grad[3 * i + 0] = gx;
          A.grad[3 * i + 1] = gy;
          A.grad[3 * i + 2] = gz;
        }
      } else {
        float f = A.L.amplitude * val;
        float fx = A.L.amplitude * gx, fy = A.L.amplitude * gy, fz = A.L.amplitude * gz;
        if (A.B.sphere) {
          const float dx = x - cx, dy = y - cy;
          const float r = sqrtf(fmaf(dx, dx, fmaf(dy, dy, z * z)));
          f = fmaf(A.L.amplitude, val, r - A.B.r0);
          if (r > 0.f) {
            fx += dx / r;
            fy += dy / r;
            fz += z / r;
          }
        }
        if (A.value) A.value[i] = f;
        if (A.grad) {
          A.grad[3 * i + 0] = fx;
          A.grad[3 * i + 1] = fy;
          A.grad[3 * i + 2] = fz;
        }
      }
    }
  }
}

// ------------------------------------------------------------------ launchers

hipError_t launch_zero_ints(int* p, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_ints, dim3((count + 255) / 256), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

hipError_t launch_queue_order(const QueueOrderArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_queue_order, dim3(grid), dim3(kOrderThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_trace_level(int width, int prec, const TraceLevelArgs& a, int grid, hipStream_t s) {
#define CALL(H, P) hipLaunchKernelGGL((k_trace_level<H, P, trace_pair(H, P)>), dim3(grid), dim3(kBlockThreads), 0, s, a)
  NNM_DISPATCH(width, prec, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_normal(int width, int prec, const NormalArgs& a, int grid, hipStream_t s) {
#define CALL(H, P) hipLaunchKernelGGL((k_normal<H, P>), dim3(grid), dim3(kBlockThreads), 0, s, a)
  NNM_DISPATCH(width, prec, CALL)
#undef CALL
  return hipGetLastError();
}

hipError_t launch_points(int width, int prec, const PointsArgs& a, int grid, hipStream_t s) {
#define CALL(H, P) hipLaunchKernelGGL((k_points<H, P>), dim3(grid), dim3(kBlockThreads), 0, s, a)
  NNM_DISPATCH(width, prec, CALL)
#undef CALL
  return hipGetLastError();
}

static int occupancy_of(const void* fn, int device) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlockThreads, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
  return per_cu * cus;
}

int resident_blocks(int width, int prec, int kind, int device) {
  int out = 0;
#define CALL(H, P)                                                                              \
  {                                                                                             \
    const void* fn = kind == 0 ? (const void*)k_trace_level<H, P, trace_pair(H, P)>             \
                               : (kind == 1 ? (const void*)k_normal<H, P> : (const void*)k_points<H, P>); \
    out = occupancy_of(fn, device);                                                             \
  }
  switch (width * 4 + prec) {
    case 32 * 4 + PREC_FP32: CALL(32, PREC_FP32); break;
    case 32 * 4 + PREC_BF16: CALL(32, PREC_BF16); break;
    case 32 * 4 + PREC_FP16: CALL(32, PREC_FP16); break;
    case 64 * 4 + PREC_FP32: CALL(64, PREC_FP32); break;
    case 64 * 4 + PREC_BF16: CALL(64, PREC_BF16); break;
    case 64 * 4 + PREC_FP16: CALL(64, PREC_FP16); break;
    case 128 * 4 + PREC_FP32: CALL(128, PREC_FP32); break;
    case 128 * 4 + PREC_BF16: CALL(128, PREC_BF16); break;
    case 128 * 4 + PREC_FP16: CALL(128, PREC_FP16); break;
    case 256 * 4 + PREC_FP32: CALL(256, PREC_FP32); break;
    case 256 * 4 + PREC_BF16: CALL(256, PREC_BF16); break;
    case 256 * 4 + PREC_FP16: CALL(256, PREC_FP16); break;
    default: out = 1;
  }
#undef CALL
  return out;
}

}  // namespace nnm

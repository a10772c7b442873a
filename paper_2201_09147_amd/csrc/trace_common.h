// trace_common.h -- device helpers shared by the tracing kernels.
#pragma once
#include "nnm_kernels.h"
#include "siren_tile.h"

namespace nnm {

// Network input of a level: (x, t) for 4-D nets, x - c(t) for nets that move
// with the centre, else x.
__device__ inline float4 net_input(const DevLevel& L, float x, float y, float z, float t, float cx, float cy) {
  if (L.d_in == 4) return make_float4(x, y, z, t);
  if (L.follow_center) return make_float4(x - cx, y - cy, z, 0.f);
  return make_float4(x, y, z, 0.f);
}

// Distance |x - c| of the base sphere, on the hardware square root (about one
// ulp; the correctly rounded software sequence costs some 20 instructions per
// evaluation on the tracing kernels' critical path).
__device__ inline float base_radius(float dx, float dy, float z) {
  return __builtin_amdgcn_sqrtf(fmaf(dx, dx, fmaf(dy, dy, z * z)));
}

__device__ inline void center_at(const DevBase& B, float t, float& cx, float& cy) {
  cx = 0.f;
  cy = 0.f;
  if (B.rho != 0.f) {
    const float tr = fract_rev(t);
    cx = B.rho * cos_rev(tr);
    cy = B.rho * sin_rev(tr);
  }
}

// One step of Algorithm 1 at one level for a live ray, given d = f_j - delta_j
// at its current point: counts the evaluation, flags d < 0, advances tau by
// step_scale d and decides the outcome: 0 keep stepping, 1 leave the level
// (d <= eps; in fixed-iteration mode after exactly fixed_iters steps, the
// final level only if |d| <= eps), 2 miss (non-finite d, tau beyond far, or
// the level's budget used).  Written with selects, not branches: every lane
// runs the same instructions.
__device__ inline int alg1_step(const TraceLevelArgs& A, float d, float& tau, int& k, int& st) {
  ++k;
  const bool fin = isfinite(d);
  const float tn = fmaf(A.step_scale, d, tau);
  const bool far_ = fin && tn > A.far;
  bool leave, budget;
  if (A.fixed_iters > 0) {  // (uniform)
    const bool end = k >= A.fixed_iters;
    const bool final_miss = A.is_final && fabsf(d) > A.eps;
    leave = end && !final_miss;
    budget = end && final_miss;
  } else {
    leave = d <= A.eps;
    budget = !leave && k >= A.max_steps;
  }
  leave = leave && fin && !far_;
  budget = budget && fin && !far_;
  st |= (fin ? 0 : ST_NONFINITE) | ((fin && d < 0.f) ? ST_NEG_STEP : 0) | (far_ ? ST_FAR : 0) |
        (budget ? ST_BUDGET : 0);
  tau = fin ? tn : tau;
  return (!fin || far_ || budget) ? 2 : (leave ? 1 : 0);
}

// A level's input queue is popped from kSegments segments at once.  Sorted
// input is laid out in runs of kOrderRun consecutive ranks dealt round-robin
// to the segments (run c to segment c mod kSegments), so every segment starts
// with its share of the longest rays and a run of neighbouring queue entries
// stays together.  segment_bounds gives segment `seg`'s entries [start,
// start + len) of a queue of n; the last run (n mod kOrderRun entries, if
// not zero) is the short one.
constexpr int kOrderRun = 64;
__device__ inline void segment_bounds(int seg, int n, int& start, int& len) {
  const int runs = (n + kOrderRun - 1) / kOrderRun;
  const int full = runs / kSegments, extra = runs - full * kSegments;
  const int last_seg = runs > 0 ? (runs - 1) % kSegments : -1;
  const int short_by = runs * kOrderRun - n;
  start = (seg * full + min(seg, extra)) * kOrderRun - (seg > last_seg ? short_by : 0);
  len = (full + (seg < extra ? 1 : 0)) * kOrderRun - (seg == last_seg ? short_by : 0);
}

// A segment of a level's input queue that may still hold entries: one
// wave-wide load of all kSegments pop counters (lane s reads segment s's, past
// the L1, since other waves move them with atomics) against each segment's
// length, then the (pick mod count)-th of the open segments, so that waves
// leaving drained segments spread over the open ones instead of all meeting
// on one counter.  -1 when every counter has passed its segment's end: the
// counters only grow, so the queue is then drained for good.  Call with all
// 64 lanes active.
__device__ inline int next_open_segment(int* heads, int n, int pick, int lane) {
  static_assert(kSegments == 64, "one segment per lane");
  int s0, len;
  segment_bounds(lane, n, s0, len);
  const int h = __hip_atomic_load(heads + lane * kHeadStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long open = __ballot(h < len);
  if (open == 0ull) return -1;
  const int k = pick % __popcll(open);
  const bool mine = ((open >> lane) & 1ull) && __popcll(open & ((1ull << lane) - 1ull)) == k;
  return __builtin_ctzll(__ballot(mine));
}

// Queue position of sorted rank r in that layout.
__device__ inline int sorted_position(int r, int n) {
  const int c = r / kOrderRun;
  int start, len;
  segment_bounds(c % kSegments, n, start, len);
  return start + (c / kSegments) * kOrderRun + (r - c * kOrderRun);
}

__device__ inline int order_key(int k) { return min(k, kOrderKeys - 1); }

// One wave's ring of finished rays and their order keys (2 kPushBatch entries
// each in LDS) published kPushBatch at a time with one atomic: the lanes of
// ballot `pmask` (the ring's lanes; this lane's position `pos`) append `ray`.
// With keys (queue_key non-null) publishing also stores each entry's key at
// its queue position and counts it in the LDS histogram `hist`.
struct PushRing {
  int start = 0, n = 0;
  __device__ inline void add(int* ring, uint8_t* ring_key, unsigned long long pmask, bool mine, int pos, int ray,
                             int key) {
    if (mine) {
      const int e = (start + n + pos) & (2 * kPushBatch - 1);
      ring[e] = ray;
      if (ring_key) ring_key[e] = (uint8_t)key;
    }
    n += __popcll(pmask);
  }
  __device__ inline void publish(int* ring, const uint8_t* ring_key, int lane, int* count, int* queue,
                                 uint8_t* queue_key, int* hist, bool all) {
    const int cnt = all ? n : kPushBatch;
    __builtin_amdgcn_wave_barrier();
    int base = 0;
    if (lane == 0) base = atomicAdd(count, cnt);
    base = __shfl(base, 0);
    if (lane < cnt) {
      const int e = (start + lane) & (2 * kPushBatch - 1);
      queue[base + lane] = ring[e];
      if (queue_key) {
        const int key = ring_key[e];
        queue_key[base + lane] = (uint8_t)key;
        atomicAdd(hist + key, 1);
      }
    }
    __builtin_amdgcn_wave_barrier();
    start = (start + cnt) & (2 * kPushBatch - 1);
    n -= cnt;
  }
};

// Instantiates CALL(H, P) for every built (width, precision) pair.
#define NNM_DISPATCH(WIDTH, PREC, CALL)                                   \
  switch ((WIDTH) * 4 + (PREC)) {                                         \
    case 32 * 4 + PREC_FP32: { CALL(32, PREC_FP32); } break;              \
    case 32 * 4 + PREC_BF16: { CALL(32, PREC_BF16); } break;              \
    case 32 * 4 + PREC_FP16: { CALL(32, PREC_FP16); } break;              \
    case 64 * 4 + PREC_FP32: { CALL(64, PREC_FP32); } break;              \
    case 64 * 4 + PREC_BF16: { CALL(64, PREC_BF16); } break;              \
    case 64 * 4 + PREC_FP16: { CALL(64, PREC_FP16); } break;              \
    case 128 * 4 + PREC_FP32: { CALL(128, PREC_FP32); } break;            \
    case 128 * 4 + PREC_BF16: { CALL(128, PREC_BF16); } break;            \
    case 128 * 4 + PREC_FP16: { CALL(128, PREC_FP16); } break;            \
    case 256 * 4 + PREC_FP32: { CALL(256, PREC_FP32); } break;            \
    case 256 * 4 + PREC_BF16: { CALL(256, PREC_BF16); } break;            \
    case 256 * 4 + PREC_FP16: { CALL(256, PREC_FP16); } break;            \
    default: return hipErrorInvalidValue;                                 \
  }

}  // namespace nnm

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

// Position of the idx-th popped entry of a level's input queue of n entries.
// The previous level appends rays in the order they finish, so the slowest
// rays of that level (grazing ones, which are also slow at this level) sit at
// the end; reading the queue backwards admits them first and shortens the
// drain tail.  Results do not depend on the order.
#ifndef NNM_QUEUE_LIFO
#define NNM_QUEUE_LIFO 1
#endif
__device__ inline int queue_slot(int idx, int n) { return NNM_QUEUE_LIFO ? n - 1 - idx : idx; }

// A level's output queue (an array of n ray ids) holds two regions: rays that
// left the level in fewer than long_steps evaluations fill it from the front,
// the others from the back.  Evaluation counts of consecutive levels are
// strongly correlated (grazing rays are slow everywhere), so the next level
// admits the back region first: the longest rays start first and the drain
// tail, the latency chain of the last rays, gets shorter.  Results do not
// depend on the order.
__device__ inline int long_slot(int idx, int n) { return n - 1 - idx; }

// One wave's ring of finished rays (2 kPushBatch entries in LDS) published
// kPushBatch at a time with one atomic: `take` lanes (ballot `pmask` over the
// ring's lanes, lane position `pos`) append `ray`.  from_back: the ring feeds
// the back region of the queue.
struct PushRing {
  int start = 0, n = 0;
  __device__ inline void add(int* ring, unsigned long long pmask, bool mine, int pos, int ray) {
    if (mine) ring[(start + n + pos) & (2 * kPushBatch - 1)] = ray;
    n += __popcll(pmask);
  }
  __device__ inline void publish(int* ring, int lane, int* count, int* queue, int qn, bool from_back, bool all) {
    const int cnt = all ? n : kPushBatch;
    __builtin_amdgcn_wave_barrier();
    int base = 0;
    if (lane == 0) base = atomicAdd(count, cnt);
    base = __shfl(base, 0);
    if (lane < cnt) {
      const int e = ring[(start + lane) & (2 * kPushBatch - 1)];
      queue[from_back ? long_slot(base + lane, qn) : base + lane] = e;
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

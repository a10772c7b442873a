// nnm_kernels.h -- kernel argument blocks and launchers of libnnm (host + device).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nnm_device.h"

namespace nnm {

// Per-ray status bits (same values as NNM_ST_* of the public header).
enum { ST_HIT = 1, ST_FAR = 2, ST_BUDGET = 4, ST_NEG_STEP = 8, ST_NONFINITE = 16 };

// One level of multiscale sphere tracing over a queue of ray ids.
struct TraceLevelArgs {
  DevLevel L;
  DevBase B;
  const float* o;
  const float* v;
  const float* t;       // may be null
  float* depth;         // carries tau between levels; +inf on a miss
  uint8_t* hit;
  float* normal;        // may be null
  uint8_t* steps;       // [n][m], may be null
  uint8_t* status;      // never null (library scratch when the caller passes null)
  const int* in_queue;  // null: ray ids 0..n-1
  const int* in_count;  // null: n
  int* in_head;         // pop counter
  int* out_queue;       // rays that finished this level (next level / hits); may be null
  int* out_count;
  int n;
  int level;
  int m;
  int is_final;
  int max_steps;
  float step_scale;
  float eps;
  float far;
  float delta;  // delta of this level; 0 on the final level
};

// Analytic normal of one level at the end points of the rays in a queue.
struct NormalArgs {
  DevLevel L;
  DevBase B;
  const float* o;
  const float* v;
  const float* t;
  const float* depth;
  float* normal;
  const int* queue;
  const int* count;
  int n;
};

// Value and gradient at arbitrary points.
struct PointsArgs {
  DevLevel L;
  DevBase B;
  const float* x;
  const float* t;
  float* value;  // may be null
  float* grad;   // may be null
  int n;
  int raw;  // 1: the network N alone; 0: the scene function f
};

hipError_t launch_zero_ints(int* p, int count, hipStream_t s);
hipError_t launch_trace_level(int width, int prec, const TraceLevelArgs& a, int grid, hipStream_t s);
hipError_t launch_normal(int width, int prec, const NormalArgs& a, int grid, hipStream_t s);
hipError_t launch_points(int width, int prec, const PointsArgs& a, int grid, hipStream_t s);
// Workgroups of each kernel kind that fit on the whole device at once.
int resident_blocks(int width, int prec, int kind, int device);  // kind: 0 trace, 1 normal, 2 points

}  // namespace nnm

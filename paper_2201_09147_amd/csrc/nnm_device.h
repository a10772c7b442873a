// nnm_device.h -- device-side network description shared by the host packer
// and the gfx950 kernels of libnnm.
//
// Tile model.  One wavefront (64 lanes) evaluates a SIREN (Eq.(2) of the paper,
// phi = sin) on a tile of 32 columns.  Lane l owns column n = l % 32 and half
// g = l / 32.  Every layer's pre-activations live in the accumulator layout of
// the 32x32 MFMA: for row block mb (32 neurons) a lane holds the 16 rows
//     row(mb, g, r) = 32 mb + 8 (r / 4) + 4 g + (r % 4),   r = 0..15,
// so one layer's outputs are the next layer's B operand without leaving the
// registers; the K order this implies is baked into the packed weights.
//
// Columns are either 32 independent points (forward-only) or 8 points with
// four columns each [h | G_x G_y G_z] (forward plus the three tangent columns
// of the analytic normal, Alg. 2 with one shared forward).
//
// Sine layers run in revolutions: W_0..W_{K-1} and b_0..b_{K-1} are packed
// divided by 2 pi, so v_sin_f32 / v_cos_f32 (which take revolutions) apply
// directly; the tangent columns carry the 2 pi back explicitly.
#pragma once
#include <stdint.h>

namespace nnm {

enum { PREC_FP32 = 0, PREC_BF16 = 1, PREC_FP16 = 2 };

constexpr int kMaxLevels = 8;
constexpr int kMaxSine = 8;
constexpr int kWaveCols = 32;       // columns per wave tile
constexpr int kBlockThreads = 256;  // 4 waves per workgroup
constexpr int kChunk = 256;         // most queue entries a wave takes per atomic
constexpr int kPushBatch = 64;      // queue entries a wave publishes per atomic
constexpr int kSegments = 64;       // input queue segments, each with its own head
constexpr int kHeadStride = 32;     // ints between segment heads (one 128-byte line each)
// Order keys of a level's output queue: min(evaluations at the level, 63).
// The next level admits rays in decreasing key order (the evaluation counts of
// consecutive levels correlate, so its longest rays start first).
constexpr int kOrderKeys = 64;
constexpr int kPipeGroups = 5;       // slot groups in flight in a weight-stationary workgroup
#ifndef NNM_WS_TRACE_COLS
#define NNM_WS_TRACE_COLS 32           // columns (rays) of a weight-stationary tracing tile
#endif
constexpr int kWsRaysPerBlock = kPipeGroups * NNM_WS_TRACE_COLS;  // ray slots of a weight-stationary tracing workgroup
constexpr int kWsPointsPerBlock = 80; // point slots of a weight-stationary normal workgroup

// Index of the accumulator-layout slot (mb, g, r) in a [H] array.
__host__ __device__ inline int acc_slot(int mb, int g, int r) { return (mb * 2 + g) * 16 + r; }
__host__ __device__ inline int acc_row(int mb, int g, int r) { return 32 * mb + 8 * (r / 4) + 4 * g + (r % 4); }

// Input neuron feeding k-slot e of lane half g at k-step ks (bf16/fp16 32x32x16).
__host__ __device__ inline int kperm_16(int ks, int g, int e) {
  return 32 * (ks / 2) + 8 * (2 * (ks % 2) + e / 4) + 4 * g + (e % 4);
}
// Input neuron feeding lane half g at k-step ks (fp32 32x32x2).
__host__ __device__ inline int kperm_2(int ks, int g) {
  const int mb = ks / 16, r = ks % 16;
  return 32 * mb + 8 * (r / 4) + 4 * g + (r % 4);
}

// Layer-0 A operand (32x32x2 fp32): for k-step ks (0..2), row block mb and lane
// l = i + 32 g: [W_0 | b_0][32 mb + i][2 ks + g] / 2pi over the augmented input
// columns (x, y, z, 1) or (x, y, z, t, 1, 0); zero past the last column.
__host__ __device__ inline int a0_index(int ks, int mb, int lane, int MB) { return (ks * MB + mb) * 64 + lane; }

struct DevLevel {
  const float* a0;    // [3][H/32][64] layer-0 A operand (see a0_index)
  const float* bh;    // [(K-1) H] acc layout: hidden biases / 2pi
  const float* wk;    // [H] acc layout: output weights (unscaled)
  const void* ah;     // packed MFMA A fragments of the hidden layers
  long long ah_stride;  // bytes per hidden layer of `ah`
  float bk;           // output bias (used when bk_dev is null)
  const float* bk_dev;  // device copy of the output bias, or null
  float amplitude;
  float delta;
  int d_in;
  int width;
  int n_sine;
  int follow_center;
  int reduce_hidden;  // 1: reduce hidden sine arguments with fract first
  float l0_safe;      // inputs with inf-norm <= l0_safe keep every layer-0 sine argument
                      // within 63 revolutions (no reduction); < 0: always reduce
  // Weight-stationary layout (width 256, two hidden layers, bf16/fp16), or null:
  const float* ws_a0;     // [4 waves][2 row blocks][3 k-steps][64 lanes] layer-0 A / 2pi
  const void* ws_ah;      // [2 layers][4 waves][2 row blocks][16 k-steps][64 lanes] 16-byte A fragments
  const float* bh_plain;  // [2][256] hidden biases / 2pi, row order
  const float* wk_plain;  // [256] output weights, row order
};

struct DevBase {
  int sphere;
  float r0;
  float rho;
};

}  // namespace nnm

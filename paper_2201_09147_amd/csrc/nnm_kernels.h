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
  const int* in_count;  // entries of in_queue; null: n
  int* in_heads;        // kSegments pop counters, kHeadStride ints apart, zeroed
  int* out_queue;       // rays that finished this level (next level / hits); may be null
  int* out_count;       // entries appended to out_queue
  uint8_t* out_key;     // [n] order key of each out_queue entry (same position); null: none
  int* out_hist;        // [kOrderKeys] entries pushed per key, zeroed; with out_key
  int n;
  int level;
  int m;
  int is_final;
  int max_steps;
  float step_scale;
  float eps;
  float far;
  float delta;  // delta of this level; 0 on the final level
  int fixed_iters;  // > 0: fixed-iteration mode, exactly this many steps at this level
};

// Reorders a level's output queue by decreasing order key (a counting sort on
// the per-key totals the level accumulated) into the segment layout the next
// level pops: runs of consecutive ranks dealt round-robin to the segments, so
// every segment holds its share of the longest rays at its front.
struct QueueOrderArgs {
  const int* in;        // unsorted queue
  const int* count;     // its entries (device)
  const uint8_t* key;   // order key of each entry of `in`
  const int* hist;      // [kOrderKeys] entries per key
  int* fill;            // [kOrderKeys] reservation counters, zeroed
  int* out;             // sorted queue (same count)
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
  const float* x;  // non-null: points mode, the point of entry i is x[3 i] (o, v, depth unused)
};

// Scene-function values at the nodes of a res^3 grid over [lo, hi]^3 (node
// (i, j, k) at index (k res + j) res + i, coordinate lo + (hi - lo) i / (res - 1)).
struct GridArgs {
  DevLevel L;
  DevBase B;
  int res;
  int n;  // res^3
  float lo, hi;
  float t;  // time of every node (4-D nets, moving base)
  float* values;
};

// Marching tetrahedra over a grid of values (count, block-sum scan, vertices, triangles).
struct MeshArgs {
  const float* values;
  int res;
  int n_nodes;
  int n_blocks;       // extraction workgroups (mesh_blocks(res))
  float lo, hi, iso;
  int* bsum_v;        // [n_blocks] vertices per block, then their exclusive prefix
  int* bsum_t;        // [n_blocks] triangles per block, then their exclusive prefix
  int* gsum_v;        // [n_groups] prefix of vertices per group of 1024 blocks
  int* gsum_t;        // [n_groups] the same for triangles
  int n_groups;       // ceil(n_blocks / 1024), at most 1024
  int* vert_off;      // [n_nodes] id of the first vertex on the node's edges (surface nodes only)
  uint8_t* mask;      // [n_nodes] inside bits of the node's 8 cube corners (outside corners copy corner 0)
  float* verts;       // [max_v][3]
  int* tris;          // [max_t][3]
  long long max_v, max_t;
  long long* counts;  // [2] total vertices, total triangles
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
  int x_stride;  // floats per point in x: 3, or 4 with the time in x[3]
};

// Device packing of flat float32 parameters for the fitting kernels.
struct FitPackArgs {
  const float* params;
  int d_in, width, n_sine;
  long long w_off[kMaxSine + 1];
  long long b_off[kMaxSine + 1];
  float* a0;    // [3][H/32][64] layer-0 A operand / 2pi
  float* bh;    // [(K-1) H] hidden biases / 2pi, accumulator layout
  float* wk;    // [H] output weights, accumulator layout
  float* ah;    // [(K-1)][H*H] hidden W / 2pi, fp32 32x32x2 fragments
  float* aht;   // [(K-1)][H*H] hidden W^T (unscaled), same fragment layout
  float4* w0t;  // [H] W_0 rows (unscaled), accumulator layout
  float* bk;    // [1] output bias
};

// Fused forward + adjoint + reverse over a batch of points.
struct FitArgs {
  DevLevel L;
  const float* aht;
  const float4* w0t;
  int n;        // points
  int n_surf;   // loss mode: points [0, n_surf) are surface samples
  int mode;     // 0: eikonal fitting loss, 1: upstream adjoints
  const float* x0;  // loss: surface points [n_surf][3]; upstream: all points [n][d_in]
  const float* x1;  // loss: uniform points [n - n_surf][3]
  const float* surf_n;
  const float* unif_sdf;
  const float* dvalue;  // upstream dL/dN [n] or null
  const float* dgrad;   // upstream dL/d grad N [n][3] or null
  float inv_ns, inv_nu;
  float* ws_abar;  // [K][Kc][H]: pre-activations, then [abar | dAbar]
  float* ws_x;     // [K][Kc][H]: inputs of layers 1..K
  float* adj;      // [Kc]: dL/dN or dL/d grad N per column
  float* loss_part;  // [waves][4] or null
  float* dx;         // [n][d_in] or null
  long long Kc;      // 4 columns per point, 32 per tile of 8 points
};

struct FitVecArgs {
  long long Kc;
  int n, n_surf, mode, d_in;
  const float* x0;
  const float* x1;
  float* mask;  // [Kc] 1 on primal columns of live points
  float* wvec;  // [d_in][Kc] column weights of the layer-0 gradient
};

hipError_t launch_fit_pack(const FitPackArgs& a, hipStream_t s);
hipError_t launch_fit_fb(const FitArgs& a, int grid, hipStream_t s);
hipError_t launch_fit_vectors(const FitVecArgs& a, hipStream_t s);
hipError_t launch_fit_loss_reduce(const float* part, int nwaves, float inv_ns, float inv_nu, float* loss4,
                                  hipStream_t s);
hipError_t launch_adam(float* params, const float* grad, float* m, float* v, long long n, float lr, float b1,
                       float b2, float eps, float bc1, float bc2, hipStream_t s);
int fit_fb_grid(int width, int device);

// Destinations of a column reduction: row `row` of vector r goes to ptr[r][row * stride[r]].
struct ColDst {
  float* ptr[5];
  long long stride[5];
};
// Column reductions run in two passes; the first writes colreduce_blocks(.) * R * H
// partial sums (kColBlocks * R * H at most) and the masked sum kSumBlocks.
constexpr int kColBlocks = 1024;
constexpr int kSumBlocks = 256;
int colreduce_blocks(long long ncols, int H);
// R weighted column sums of the columns col = j * cstep of a [Kc][H] slab.
hipError_t launch_colreduce(const float* M, int H, long long Kc, const float* w, int R, int cstep, float* part,
                            const ColDst& dst, hipStream_t s);
hipError_t launch_wgrad(int H, const float* abar, const float* X, long long Kc, int chunk, float* part, float* dst,
                        hipStream_t s);
hipError_t launch_masked_sum(const float* a, const float* m, long long n, int cstep, float* part, float* out,
                             hipStream_t s);

hipError_t launch_zero_ints(int* p, int count, hipStream_t s);
hipError_t launch_box_points(uint64_t seed, long long base, int count, float lo, float hi, float* x, float* t,
                             hipStream_t s);
hipError_t launch_ref_sdf(const float* x, int count, int kind, float a, float b, float* out, hipStream_t s);
hipError_t launch_absdiff_max(const float* fa, const float* fb, int count, unsigned int* out, hipStream_t s);
hipError_t launch_trace_level(int width, int prec, const TraceLevelArgs& a, int grid, hipStream_t s);
hipError_t launch_queue_order(const QueueOrderArgs& a, int grid, hipStream_t s);
hipError_t launch_normal(int width, int prec, const NormalArgs& a, int grid, hipStream_t s);
hipError_t launch_points(int width, int prec, const PointsArgs& a, int grid, hipStream_t s);
hipError_t launch_trace_ws(int prec, const TraceLevelArgs& a, int grid, hipStream_t s);
hipError_t launch_normal_ws(int prec, const NormalArgs& a, int grid, hipStream_t s);
int ws_resident_blocks(int prec, int kind, int device);  // kind: 0 trace, 1 normal
hipError_t launch_grid_values(int width, int prec, const GridArgs& a, int device, hipStream_t s);
constexpr int kMeshThreads = 256;  // threads of an extraction workgroup
int mesh_blocks(int res);          // workgroups of the flat extraction passes for a grid side
hipError_t launch_marching_tets(const MeshArgs& a, hipStream_t s);
// Workgroups of each kernel kind that fit on the whole device at once.
int resident_blocks(int width, int prec, int kind, int device);  // kind: 0 trace, 1 normal, 2 points

}  // namespace nnm

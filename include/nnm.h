/*
 * nnm.h -- C ABI of libnnm: sphere tracing of nested sinusoidal-MLP (SIREN)
 * signed distance functions on AMD Instinct MI355X (gfx950), after da Silva et
 * al., "Neural Implicit Mapping via Nested Neighborhoods".
 *
 * Conventions for every entry point:
 *   - Return value: NNM_OK (0) or a negative NNM_E_* code; nnm_last_error()
 *     returns a thread-local message for the last failure.  Argument and
 *     descriptor validation happens before anything is enqueued, so a failed
 *     call never writes partial output.
 *   - Arrays named "device" are caller-owned device memory on the stack's
 *     device; the library never frees them.  Arrays named "host" are read
 *     during the call only.
 *   - Calls that take a stream (a hipStream_t passed as void*; NULL is the
 *     null stream) are asynchronous on that stream.  Device faults surface on a
 *     later call or on nnm_sync().
 *   - n == 0 is a no-op returning NNM_OK.
 *   - Levels are 0-based.  Points and directions are [n][3] float32 row major.
 */
#ifndef NNM_H
#define NNM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
#define NNM_OK 0
#define NNM_E_INVAL (-1)       /* null pointer, bad level, n < 0, bad parameter */
#define NNM_E_FORMAT (-2)      /* malformed network file or descriptor shape */
#define NNM_E_NONFINITE (-3)   /* NaN or Inf in weights, amplitudes or deltas */
#define NNM_E_LIPSCHITZ (-4)   /* Lipschitz bound of a level exceeds lipschitz_max */
#define NNM_E_NESTING (-5)     /* deltas not strictly decreasing and positive */
#define NNM_E_NOMEM (-6)       /* host or device allocation failed */
#define NNM_E_DEVICE (-7)      /* HIP runtime error (launch, copy, fault) */
#define NNM_E_UNSUPPORTED (-8) /* width / input size / precision not built */
#define NNM_E_IO (-9)          /* file could not be read */

/* Precision of the hidden (width x width) layers.  The first layer, the sine
   argument reduction, the biases, the output layer and the scene terms always
   run in float32; products accumulate in float32. */
#define NNM_PREC_FP32 0
#define NNM_PREC_BF16 1
#define NNM_PREC_FP16 2

/* Per-ray status bits written by trace_rays. */
#define NNM_ST_HIT 1        /* the last traced level reached d <= eps */
#define NNM_ST_FAR 2        /* the ray parameter passed far: a miss */
#define NNM_ST_BUDGET 4     /* a level used max_steps evaluations: a miss */
#define NNM_ST_NEG_STEP 8   /* some step had d < 0 (start inside a band) */
#define NNM_ST_NONFINITE 16 /* a non-finite scene value: a miss */

/* ------------------------------------------------------------ descriptors */

/* One network of the nested sequence with its scene terms (Sec. 3.2, Eq.(1)):
     f_j(x, t) = [|x - c(t)| - r0] + amplitude * N_j(input)
   with input = x, x - c(t) (follow_center) or (x, t) for d_in == 4, and N_j the
   MLP of Eq.(2), N(p) = W_K h_K + b_K, h_0 = p, h_{i+1} = sin(W_i h_i + b_i).
   params: host float32, W_0, b_0, W_1, b_1, ..., W_K, b_K, each W_i row major
   [out][in]; shapes [width][d_in], [width][width] (K - 1 times), [1][width].
   omega0 of the SIREN first layer must already be folded into W_0, b_0. */
typedef struct {
  int32_t d_in;          /* 3 (x, y, z) or 4 (x, y, z, t) */
  int32_t width;         /* 32, 64, 128 or 256 */
  int32_t n_sine;        /* K sine layers (1 .. 8) */
  int32_t follow_center; /* 1: the net input is x - c(t) */
  float amplitude;       /* scale of the network term (finite) */
  float delta;           /* threshold delta_j of the nesting condition; ignored
                            on the last level of the sequence */
  const float* params;   /* host, see above */
} nnm_level_desc;

/* A nested sequence f_1 |> ... |> f_m (Sec. 3.2) and its common base term. */
typedef struct {
  int32_t n_levels;      /* m, 1 .. 8 */
  int32_t base_sphere;   /* 1: include |x - c(t)| - r0 in every f_j */
  float r0;              /* sphere radius */
  float rho;             /* c(t) = rho (cos 2 pi t, sin 2 pi t, 0); 0: static */
  float lipschitz_max;   /* reject a level whose bound 1 + a * prod_i sigma(W_i)
                            (spatial columns of W_0; 0 + ... without the sphere)
                            exceeds this; 0 disables the check */
  int32_t reserved;
  const nnm_level_desc* levels; /* host, n_levels entries */
} nnm_stack_desc;

typedef struct nnm_stack nnm_stack; /* opaque; immutable after loading */

/* Multiscale sphere tracing parameters (Algorithm 1, Sec. 4).  Per level j the
   tracer repeats: d = f_j(o + tau v) - delta_j (delta = 0 on final_level);
   tau += step_scale * d; then tau > far -> miss; d <= eps -> next level;
   max_steps evaluations used -> miss.
   mode 1 is fixed-iteration tracing (the paper's experiments fix the iteration
   counts, Sec. 6 and Table 3): level j <= final_level takes exactly
   iterations[j] steps (1..255) with no eps exit; tau > far is still a miss;
   after the final level a ray is a hit iff its last |d| <= eps (else a miss
   flagged NNM_ST_BUDGET).  max_steps is unused in mode 1. */
#define NNM_MAX_LEVELS 8
typedef struct nnm_profiler nnm_profiler; /* see "profiling" below */

/* Kernel family of trace_rays.  Both compute the same Algorithm 1 and normals;
   they differ in the order of the float32 sums inside a layer.
   AUTO: the pipelined weight-stationary kernels on the levels that have them
   (width 256, two hidden layers, bf16/fp16), the streaming tile elsewhere.
   STREAMING: the streaming tile on every level. */
#define NNM_KERNELS_AUTO 0
#define NNM_KERNELS_STREAMING 1

typedef struct {
  float step_scale;      /* s, in (0, 1] */
  float eps;             /* eps > 0 */
  float far;             /* far > 0 */
  int32_t max_steps;     /* evaluations per level, 1 .. 255 */
  int32_t final_level;   /* last traced level (m - 1: full; m - 2: NNM) */
  int32_t normal_level;  /* level whose unit gradient is returned as the normal;
                            > final_level is neural normal mapping (Sec. 5) */
  int32_t mode;          /* 0: eps-terminated; 1: fixed iterations per level */
  int32_t kernels;       /* NNM_KERNELS_AUTO or NNM_KERNELS_STREAMING */
  nnm_profiler* profiler; /* NULL, or a profiler that times every kernel of the call */
  int32_t iterations[NNM_MAX_LEVELS]; /* mode 1: steps of each traced level */
} nnm_trace_params;

/* ---------------------------------------------------------------- stacks */

/* Validates a stack descriptor on the host only (no device use): shapes and
   supported sizes (NNM_E_UNSUPPORTED / NNM_E_FORMAT), finiteness
   (NNM_E_NONFINITE), deltas of levels 0 .. m-2 strictly decreasing and > 0
   (NNM_E_NESTING) and the Lipschitz bound (NNM_E_LIPSCHITZ). */
int nnm_validate_stack(const nnm_stack_desc* desc, int precision);

/* The Lipschitz product bound of one level (power iteration in float64 on the
   host): amplitude * sigma(W_0[:, 0:3]) * prod_{i>=1} sigma(W_i), plus 1 when
   base_sphere.  Returns NNM_OK and writes *bound. */
int nnm_level_lipschitz_bound(const nnm_level_desc* level, int base_sphere, double* bound);

/* Loads a nested sequence f_1 |> ... |> f_m (Sec. 3.2: each level a neural SDF
   whose delta_j-neighbourhood contains the next level's, Eq.(1); each network
   the sine MLP of Eq.(2), Sec. 5.1) for tracing on `device`.
   Validates desc as nnm_validate_stack does (nothing is allocated on a
   failure), packs the weights for `precision` (float32 masters; bf16 / fp16
   copies of the hidden layers, rounded to nearest even) and uploads them
   once.  The descriptor and its parameter arrays may be freed afterwards.
   *out is owned by the caller and released with free_siren_stack; a loaded
   stack is immutable, so calls on several streams may share it.
   Errors: NNM_E_INVAL (null out, bad device), the validation codes,
   NNM_E_NOMEM, NNM_E_DEVICE. */
int load_siren_stack(const nnm_stack_desc* desc, int precision, int device, nnm_stack** out);

/* Frees the library-owned device copies of a stack; NULL is a no-op. */
void free_siren_stack(nnm_stack* stack);

/* Number of levels and precision of a loaded stack (NULL -> -1). */
int nnm_stack_levels(const nnm_stack* stack);
int nnm_stack_precision(const nnm_stack* stack);

/* ---------------------------------------------------------------- tracing */

/* Multiscale sphere tracing of n rays (Algorithm 1) with the analytic normal of
   level normal_level at the end point (Sec. 5.1; neural normal mapping when
   normal_level > final_level, Sec. 5).
     o, v    device [n][3] float32; v of unit length
     t       device [n] float32 times, or NULL (t = 0)
     depth   device [n] float32 out: ray parameter tau of the end point; +inf on a miss
     hit     device [n] uint8 out: 1 hit, 0 miss
     normal  device [n][3] float32 out: unit grad f_normal_level at o + tau v
             (0 on a miss), or NULL to skip the normal pass
     steps   device [n][m] uint8 out: evaluations per level (0 for levels not
             reached), or NULL
     status  device [n] uint8 out: NNM_ST_* bits, or NULL
   Uses stream-ordered scratch (ray queues and counters) of about 9 n bytes. */
int trace_rays(const nnm_stack* stack, const nnm_trace_params* params, int64_t n, const float* o,
               const float* v, const float* t, float* depth, uint8_t* hit, float* normal,
               uint8_t* steps, uint8_t* status, void* stream);

/* Largest n that trace_rays_noalloc accepts (a 1920 x 1080 frame fits). */
#define NNM_NOALLOC_MAX_RAYS (1 << 21)

/* trace_rays for callers that cannot allocate: code under HIP graph capture,
   tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
   kernels and results as trace_rays, but it calls no hipMalloc, hipFree or
   allocating routine: its scratch (ray queues, order keys, counters, status carrier;
   about 21 MB) is a static device array of the library, one per GPU, which
   each GPU the library runs on holds until the process ends.  Its address is
   looked up on the first call on a device.
   Every call on one GPU uses that GPU's one array: calls that may overlap in
   time on one GPU (other streams, other threads, no ordering between them)
   race and give wrong results; calls on one stream are ordered and safe.
   Errors: those of trace_rays; NNM_E_INVAL for n > NNM_NOALLOC_MAX_RAYS or a
   non-NULL params->profiler (a profiler creates events); NNM_E_DEVICE when
   the array's address cannot be looked up. */
int trace_rays_noalloc(const nnm_stack* stack, const nnm_trace_params* params, int64_t n,
                       const float* o, const float* v, const float* t, float* depth, uint8_t* hit,
                       float* normal, uint8_t* steps, uint8_t* status, void* stream);

/* Analytic gradient of one scene function (Eq.(3)-(4) with the G_i form of
   Alg. 2, one shared forward for the three tangent columns):
     x      device [n][3] points; t device [n] or NULL
     value  device [n] out: f_level(x, t), or NULL
     grad   device [n][3] out: raw grad_x f_level (not normalised) */
int analytic_normal(const nnm_stack* stack, int level, int64_t n, const float* x, const float* t,
                    float* value, float* grad, void* stream);

/* The raw network N_level and its spatial gradient (no scene terms, no
   amplitude): value device [n] (or NULL), grad device [n][3] (or NULL). */
int nnm_net_eval(const nnm_stack* stack, int level, int64_t n, const float* x, const float* t,
                 float* value, float* grad, void* stream);

/* ---------------------------------------------------------------- fitting */

/* Differentiation of one SIREN N (Eq.(2)) with respect to its parameters,
   through the value and the analytic gradient (a double backward), in
   float32.  `params` is the flat float32 parameter vector in nnm_level_desc
   order; `d_in` 3 or 4 (the gradient is w.r.t. the first three inputs), width
   32 / 64 / 128 / 256, 1 .. 8 sine layers. */
typedef struct {
  int32_t d_in;
  int32_t width;
  int32_t n_sine;
  int32_t reserved;
} nnm_net_shape;

/* Bytes of device workspace that siren_backward needs for n points. */
int64_t siren_workspace_bytes(const nnm_net_shape* shape, int64_t n);

/* Forward with tangents: value[n] = N(x), grad[n][3] = grad_x N (either may
   be NULL).  params, x: device.  No workspace; asynchronous on `stream`. */
int siren_forward_tangent(const nnm_net_shape* shape, const float* params, int64_t n, const float* x,
                          float* value, float* grad, void* stream);

/* Reverse mode through primal and tangent: given upstream adjoints
   dvalue[n] (= dL/dN, may be NULL for 0) and dgrad[n][3] (= dL/d grad N, may be
   NULL for 0), writes dparams[P] (= dL/dparams, overwritten) and, if dx is not
   NULL, dx[n][d_in] (= dL/dx through N only).  The forward is recomputed; the
   workspace (device, >= siren_workspace_bytes) holds per-layer values for the
   weight-gradient products.  All pointers device; asynchronous on `stream`. */
int siren_backward(const nnm_net_shape* shape, const float* params, int64_t n, const float* x,
                   const float* dvalue, const float* dgrad, float* dparams, float* dx, void* workspace,
                   int64_t workspace_bytes, void* stream);

/* A fitting state: parameters, Adam moments and step counter on one device,
   with the workspace for up to max_points points per step. */
typedef struct nnm_fit nnm_fit;

/* One batch of the eikonal fitting loss (device pointers):
     L = mean_surf |N| + mean_surf (1 - n . grad N / |grad N|)
       + mean_unif |N - sdf| + mean_unif (|grad N| - 1)^2
   (the normal term compares the unit gradient with n; it is 1 where
   grad N = 0). */
typedef struct {
  int64_t n_surf;
  int64_t n_unif;
  const float* surf_x;   /* [n_surf][3] points on the surface */
  const float* surf_n;   /* [n_surf][3] unit normals there */
  const float* unif_x;   /* [n_unif][3] points in the domain */
  const float* unif_sdf; /* [n_unif] signed distances there */
} nnm_fit_batch;

/* Adam (Kingma & Ba, bias corrected, no weight decay). */
typedef struct {
  float lr;
  float beta1;
  float beta2;
  float eps;
} nnm_adam;

/* Creates a fitting state from host float32 parameters (copied). */
int fit_create(const nnm_net_shape* shape, const float* params, int device, int64_t max_points, nnm_fit** out);
void fit_free(nnm_fit* fit);

/* One step of fitting a neural SDF (Sec. 3.3, "MLPs for a single surface":
   each network is trained to a known SDF with the eikonal approach the paper
   cites; the loss terms are those of nnm_fit_batch, with the normal term on
   the unit gradient): the loss, its parameter gradient by reverse mode through
   the value and the analytic gradient of Sec. 5.1 (a double backward), and an
   Adam update.  batch: device arrays of at most max_points points in total;
   loss4: device [4] out (the four mean terms), or NULL.  Asynchronous on
   `stream`.  Every sum over points runs over a fixed partition in a fixed
   order, so the same state and batch give bitwise the same step on the same
   device.  Errors: NNM_E_INVAL (null, a negative count, more than max_points
   points, lr or eps not positive, a beta outside [0, 1)),
   NNM_E_UNSUPPORTED (a 4-D network: the loss takes 3-D points), NNM_E_DEVICE. */
int fit_step(nnm_fit* fit, const nnm_fit_batch* batch, const nnm_adam* opt, float* loss4, void* stream);

/* Loss terms and gradient only (no update): dparams device [P] out. */
int fit_loss_grad(nnm_fit* fit, const nnm_fit_batch* batch, float* loss4, float* dparams, void* stream);

/* Device pointers of the state (owned by the fit; valid until fit_free):
   params, Adam first and second moments, each [P] float32. */
int fit_state(nnm_fit* fit, float** params, float** adam_m, float** adam_v, int64_t* n_params);
/* Copies params, Adam m and v to host arrays of n_params floats (any may be
   NULL); synchronises the device.  A checkpoint together with fit_get_step. */
int fit_read_state(nnm_fit* fit, float* params, float* adam_m, float* adam_v);
/* Writes the current parameters as a network file (nnm_write_net_file), the
   input of load_siren_stack after a fit (the fitted network of the torus
   workload is rendered this way).  Synchronises the fit's device first.
   Errors: NNM_E_INVAL, NNM_E_NOMEM, NNM_E_DEVICE, NNM_E_IO. */
int fit_export(nnm_fit* fit, const char* path);
/* Overwrites params, m, v from host arrays (any may be NULL); synchronous. */
int fit_write_state(nnm_fit* fit, const float* params, const float* adam_m, const float* adam_v);
/* Steps taken so far (Adam's t); settable for a resumed run. */
int64_t fit_get_step(const nnm_fit* fit);
int fit_set_step(nnm_fit* fit, int64_t step);

/* ------------------------------------------------------ nesting thresholds */

/* Sampled infinity norm of f_a - f_b, the scene functions of two levels of a
   stack, over the box [lo, hi]^3 (and t in [0, 1) when a level is 4-D or the
   base moves): Sec. 3.3 approximates |f|_inf by a maximum over sampled
   points, and Proposition 1 turns such bounds into nesting thresholds
   (nnm_nesting_thresholds).  n points are drawn by splitmix64 from seed:
   stream position k = 4 i + c for coordinate c of point i, u = (z >> 40) / 2^24,
   x_c = float(lo + (hi - lo) u) evaluated in double, t = float(u) of c = 3.
   out_max: one device float, overwritten (a NaN difference gives +inf).
   Asynchronous on `stream`; allocates a stream-ordered scratch of about 24 MB.
   Errors: NNM_E_INVAL (null, bad level, n < 1, empty box), NNM_E_NOMEM,
   NNM_E_DEVICE. */
int nnm_sup_abs_diff(const nnm_stack* s, int level_a, int level_b, int64_t n, uint64_t seed, float lo, float hi,
                     float* out_max, void* stream);

/* A known signed distance function f, the target that the networks of
   Proposition 2 approximate ("MLPs for a single surface", Sec. 3.3), evaluated
   in float32:
     NNM_REF_SPHERE  |x| - a
     NNM_REF_TORUS   sqrt((sqrt(x^2 + y^2) - a)^2 + z^2) - b  (axis z, major
                     radius a, minor radius b) */
#define NNM_REF_SPHERE 1
#define NNM_REF_TORUS 2
typedef struct {
  int32_t kind; /* NNM_REF_SPHERE or NNM_REF_TORUS */
  float a;      /* radius (sphere) or major radius (torus), > 0 */
  float b;      /* minor radius (torus), > 0; unused for the sphere */
  int32_t reserved;
} nnm_ref_sdf;

/* Sampled infinity norm of f - f_level: the scene function of one level
   against a known SDF, over the same splitmix64 points as nnm_sup_abs_diff
   (same seed, same n, same box give the same points).  The bound
   |f - f_theta_i|_inf < eps_i that Proposition 2 turns into thresholds.
   out_max: one device float, overwritten (a NaN difference gives +inf).
   Asynchronous on `stream`; stream-ordered scratch of about 24 MB.
   Errors: NNM_E_INVAL (null, bad level, n < 1, empty box, unknown shape or
   non-positive radius), NNM_E_NOMEM, NNM_E_DEVICE. */
int nnm_sup_abs_err(const nnm_stack* s, int level, const nnm_ref_sdf* ref, int64_t n, uint64_t seed, float lo,
                    float hi, float* out_max, void* stream);

/* Nesting thresholds from bounds on infinity norms (Sec. 3.3, Propositions 1
   and 2).  Host only, float64, no device use.  Each bound becomes
   eps_i = sup[i] + margin: the propositions need strict bounds
   (eps_i > |.|_inf), and a sampled maximum approaches the supremum from below,
   so margin (>= 0) is the caller's allowance for that.  0-based levels:
     NNM_NEST_PROP1  consecutive members, sup[i] >= |f_i - f_{i-1}|_inf for
                     i = 1 .. m-1 (sup[0] is not read):
                       delta[m-1] = eps_{m-1},
                       delta[i-1] = delta[i] + eps_i          (i = m-1 .. 1)
     NNM_NEST_PROP2  members approximating one SDF f, sup[i] >= |f - f_i|_inf
                     for i = 0 .. m-1:
                       delta[m-1] = eps_{m-1} + eps_{m-2},
                       delta[i-1] = delta[i] + eps_i + eps_{i-1}  (i = m-1 .. 1)
   Writes delta[0 .. m-1]; trace_rays reads delta[0 .. m-2] (the level
   descriptors' delta) and traces the last level to its zero set.
   Errors: NNM_E_INVAL (null, m outside 2 .. NNM_MAX_LEVELS, unknown
   proposition, a negative or non-finite bound or margin). */
#define NNM_NEST_PROP1 1
#define NNM_NEST_PROP2 2
int nnm_nesting_thresholds(int proposition, int32_t m, const double* sup, double margin, double* delta);

/* ------------------------------------------- neural normal mapping on meshes */

/* Neural normal mapping onto arbitrary points, e.g. the vertices of a triangle
   mesh (Sec. 5: the detailed normals of a finer scene function are assigned to
   the vertices of a coarser surface, with no parametrisation):
     x       device [n][3] float32 points; t device [n] or NULL (time 0)
     normal  device [n][3] float32 out: grad f_level / |grad f_level| (the
             analytic gradient of Sec. 5.1), 0 where the gradient vanishes.
   Same kernels and precision as the normal pass of trace_rays.  n = 0 is a
   no-op.  Errors: NNM_E_INVAL (null, bad level, n < 0 or n > 2^31 - 2^24). */
int neural_normal_map(const nnm_stack* stack, int level, int64_t n, const float* x, const float* t,
                      float* normal, void* stream);

/* Largest grid side of nnm_grid_values / nnm_mesh_extract (node, vertex and
   triangle ids then fit int32). */
#define NNM_MESH_MAX_RES 512

/* The scene function f_level at the nodes of a res^3 grid over [lo, hi]^3, the
   input of the coarse-mesh extraction (Fig. 5 extracts its coarse mesh from a
   (64,1) network):
     values  device [res^3] float32 out; node (i, j, k) at index
             (k res + j) res + i (x fastest), at coordinates
             float(lo + (hi - lo) i / (res - 1)) evaluated in double, likewise
             for j and k.
     t       time of every node (4-D levels, moving base); ignored otherwise.
   Errors: NNM_E_INVAL (null, bad level, res outside [2, NNM_MESH_MAX_RES],
   lo >= hi, non-finite box or time). */
int nnm_grid_values(const nnm_stack* stack, int level, int32_t res, float lo, float hi, float t,
                    float* values, void* stream);

/* The coarse triangle mesh {f < iso} of a grid of values by marching
   tetrahedra (the paper uses marching cubes and does not fix the variant; the
   tetrahedral form gives a closed, consistently oriented surface).  The output
   is deterministic:
     - a node is inside when value < iso (NaN is outside);
     - node (i, j, k) owns the edges to node + D for D in the order (1,0,0)
       (0,1,0) (0,0,1) (1,1,0) (1,0,1) (0,1,1) (1,1,1); an edge whose ends differ
       holds one vertex at x0 + (iso - v0) / (v1 - v0) (x1 - x0), and vertices
       are numbered in (node, edge) order;
     - the cube at node (i, j, k) (all < res - 1) holds six tetrahedra, one per
       axis order (a, b, c) in lexicographic order with corners 0, e_a,
       e_a + e_b, (1,1,1), the middle two swapped for odd orders; triangles come
       in cube order, then tetrahedron order; every triangle is wound
       counter-clockwise seen from the outside (value >= iso) side.
     values  device [res^3] float32, the layout of nnm_grid_values
     verts   device [max_verts][3] float32 out (the first max_verts vertices)
     tris    device [max_tris][3] int32 out (vertex ids; the first max_tris)
     counts  device [2] int64 out: total vertices, total triangles (also when
             they exceed the capacities; call again with larger arrays then)
   Runs on the current device.  Allocates stream-ordered scratch of about
   5 res^3 bytes.  Errors: NNM_E_INVAL (null values or counts, res outside
   [2, NNM_MESH_MAX_RES], lo >= hi, non-finite box or iso, negative capacity, a
   null array with a positive capacity), NNM_E_NOMEM, NNM_E_DEVICE. */
int nnm_mesh_extract(const float* values, int32_t res, float lo, float hi, float iso, int64_t max_verts,
                     int64_t max_tris, float* verts, int32_t* tris, int64_t* counts, void* stream);

/* -------------------------------------------------------------- profiling */

/* A profiler records a HIP event pair around every kernel that trace_rays
   launches while it is attached to the trace parameters (events on the call's
   stream; no synchronisation until a report is requested).  Entries are keyed
   by (kind, level, variant): kind 0 = tracing of one level, 1 = normal pass,
   2 = ordering of level `level`'s output queue for the next level
   (k_queue_order, variant 0); variant 0 = single-wave streaming tile
   (k_trace_level / k_normal), 1 = pipelined weight-stationary workgroup
   (k_trace_ws / k_normal_ws). */
#define NNM_PROF_MAX 32
typedef struct {
  int32_t n_entries;
  int32_t kind[NNM_PROF_MAX];
  int32_t level[NNM_PROF_MAX];
  int32_t width[NNM_PROF_MAX];
  int64_t launches[NNM_PROF_MAX];
  double total_ms[NNM_PROF_MAX];
  int32_t variant[NNM_PROF_MAX];
} nnm_profile_report;

int nnm_profiler_create(nnm_profiler** out);
void nnm_profiler_free(nnm_profiler* prof);
/* Discards recorded events. */
int nnm_profiler_reset(nnm_profiler* prof);
/* Synchronises the recorded events and sums their durations per entry. */
int nnm_profiler_report(nnm_profiler* prof, nnm_profile_report* out);

/* --------------------------------------------------------------- utilities */

/* Network file: "NNMW", u32 version 1, u32 d_in, u32 width, u32 n_sine,
   3 x u32 reserved, then the float32 parameters in nnm_level_desc order.
   On success *params_out is malloc'ed (free with nnm_free) and the shape
   fields are written.  Errors: NNM_E_IO, NNM_E_FORMAT. */
int nnm_read_net_file(const char* path, int32_t* d_in, int32_t* width, int32_t* n_sine,
                      float** params_out, int64_t* n_params);
void nnm_free(void* p);

/* Writes a network file (the format above) from host float32 parameters;
   n_params must equal nnm_param_count(d_in, width, n_sine).  The file is
   written to path + ".tmp" and renamed, so a reader never sees a partial file.
   Errors: NNM_E_INVAL (null, shape, count), NNM_E_IO. */
int nnm_write_net_file(const char* path, int32_t d_in, int32_t width, int32_t n_sine, const float* params,
                       int64_t n_params);

/* Number of float32 parameters of a network shape (< 0 if unsupported). */
int64_t nnm_param_count(int32_t d_in, int32_t width, int32_t n_sine);

/* Blocks until `stream` is idle and reports a pending device error. */
int nnm_sync(void* stream);

/* Thread-local description of the last error ("" if none). */
const char* nnm_last_error(void);

/* Library version string. */
const char* nnm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NNM_H */

/*
 * nnm_oracle.c -- plain double-precision CPU oracle for sphere tracing of nested
 * sinusoidal-MLP (SIREN) signed distance functions, after da Silva et al.,
 * "Neural Implicit Mapping via Nested Neighborhoods".
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load or call this library.  The GPU library never
 * links, loads or calls it, and it shares no code, header or table with the GPU
 * path.  It reads the same float32 weights and float32 rays as the GPU (upcast
 * exactly to double) and does all arithmetic in double precision, slowly and
 * literally:
 *
 *   net_value       N(x) = W_K h_K + b_K, h_0 = x, h_{i+1} = sin(W_i h_i + b_i)
 *                   (the MLP form of Eq.(2) with phi = sin; omega0 is folded into
 *                   W_0, b_0 by the weight generator).
 *   net_value_grad  grad N by the chain rule of Eq.(3): W_K * J_{K-1} * ... * J_0,
 *                   with each layer Jacobian formed explicitly as the matrix
 *                   J_i = W_i (Hadamard) phi'[a_i | ... | a_i] of Eq.(4) and the
 *                   product taken right to left on the three spatial columns.
 *   scene_*         f_j(x,t) = |x - c(t)| - r0 + a_j N_j(input), c(t) = rho (cos 2 pi t,
 *                   sin 2 pi t, 0); grad_x f_j = (x - c)/|x - c| + a_j grad_x N_j.
 *   trace_one       multiscale sphere tracing, Algorithm 1 (Sec. 4), with the
 *                   readings listed at that function.
 *   normals         unit grad f of the chosen normal level at the end point: the
 *                   analytic normal (Sec. 5.1) and, when the normal level is finer
 *                   than the last traced level, neural normal mapping (Sec. 5).
 *   orc_first_root  brute-force first zero crossing along a ray (a check of the
 *                   first-hit claim after Algorithm 1; not part of the method).
 *
 * Parity is pinned by the CPU tests (closed forms, complex-step and central
 * differences, the analytic sphere, brute-force roots, Lipschitz safety).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAX_LAYERS 16
#define ORC_MAX_LEVELS 8

/* Status bits of one ray. */
#define ORC_ST_HIT 1
#define ORC_ST_FAR 2
#define ORC_ST_BUDGET 4
#define ORC_ST_NEG_STEP 8
#define ORC_ST_NONFINITE 16

typedef struct {
  int d_in;          /* 3, or 4 for (x, y, z, t) */
  int width;         /* H */
  int n_sine;        /* K sine layers, K + 1 affine layers */
  int follow_center; /* input is x - c(t) */
  double amplitude;  /* a_j */
  double delta;      /* delta_j (ignored on the last traced level) */
  const float* params; /* W_0, b_0, ..., W_K, b_K; W_i row major [out][in] */
} orc_level_desc;

typedef struct {
  int d_in, width, n_sine;
  int rows[ORC_MAX_LAYERS], cols[ORC_MAX_LAYERS];
  double* W[ORC_MAX_LAYERS];
  double* b[ORC_MAX_LAYERS];
  double* store;
} orc_net;

typedef struct {
  orc_net net;
  int follow_center;
  double amplitude, delta;
} orc_level;

/* Base term of every level: |x - c(t)| - r0 when sphere != 0, else 0. */
typedef struct {
  int sphere;
  double r0;  /* sphere radius */
  double rho; /* circle radius of the centre motion c(t); 0 for a static centre */
} orc_base_desc;

static void net_free(orc_net* net) {
  free(net->store);
  net->store = NULL;
}

static int net_load(orc_net* net, int d_in, int width, int n_sine, const float* params) {
  memset(net, 0, sizeof(*net));
  if (n_sine < 1 || n_sine + 1 > ORC_MAX_LAYERS || width < 1 || d_in < 1 || !params) return -1;
  net->d_in = d_in;
  net->width = width;
  net->n_sine = n_sine;
  size_t total = 0;
  for (int i = 0; i <= n_sine; ++i) {
    net->rows[i] = (i == n_sine) ? 1 : width;
    net->cols[i] = (i == 0) ? d_in : width;
    total += (size_t)net->rows[i] * net->cols[i] + net->rows[i];
  }
  net->store = (double*)malloc(total * sizeof(double));
  if (!net->store) return -1;
  for (size_t k = 0; k < total; ++k) net->store[k] = (double)params[k];
  double* p = net->store;
  for (int i = 0; i <= n_sine; ++i) {
    net->W[i] = p;
    p += (size_t)net->rows[i] * net->cols[i];
    net->b[i] = p;
    p += net->rows[i];
  }
  return 0;
}

/* Workspace (doubles) for one evaluation with explicit Jacobians. */
static size_t net_ws_size(const orc_net* net) {
  size_t w = (size_t)(net->width > net->d_in ? net->width : net->d_in);
  return 4 * w + 6 * w + w * w;
}

/* Eq.(2): forward pass only. h, hn: buffers of max(width, d_in) doubles. */
static double net_value(const orc_net* net, const double* in, double* h, double* hn) {
  memcpy(h, in, sizeof(double) * net->d_in);
  for (int i = 0; i < net->n_sine; ++i) {
    const int R = net->rows[i], C = net->cols[i];
    for (int r = 0; r < R; ++r) {
      double a = net->b[i][r];
      for (int c = 0; c < C; ++c) a += net->W[i][(size_t)r * C + c] * h[c];
      hn[r] = sin(a);
    }
    double* tmp = h;
    h = hn;
    hn = tmp;
  }
  const int K = net->n_sine, C = net->cols[K];
  double out = net->b[K][0];
  for (int c = 0; c < C; ++c) out += net->W[K][c] * h[c];
  return out;
}

/* Eq.(2) value and Eq.(3)-(4) gradient w.r.t. the first three inputs.
   ws: net_ws_size(net) doubles. */
static double net_value_grad(const orc_net* net, const double* in, double grad[3], double* ws) {
  const size_t w = (size_t)(net->width > net->d_in ? net->width : net->d_in);
  double* h = ws;
  double* hn = h + w;
  double* a = hn + w;
  double* M = a + w;      /* running product, rows x 3 */
  double* Mn = M + 3 * w; /* next running product */
  double* J = Mn + 3 * w; /* explicit layer Jacobian */
  memcpy(h, in, sizeof(double) * net->d_in);
  /* d h_0 / d x restricted to the spatial columns: the first three unit vectors. */
  for (int c = 0; c < net->d_in; ++c)
    for (int j = 0; j < 3; ++j) M[c * 3 + j] = (c == j) ? 1.0 : 0.0;
  for (int i = 0; i < net->n_sine; ++i) {
    const int R = net->rows[i], C = net->cols[i];
    for (int r = 0; r < R; ++r) {
      double s = net->b[i][r];
      for (int c = 0; c < C; ++c) s += net->W[i][(size_t)r * C + c] * h[c];
      a[r] = s;
    }
    /* Eq.(4): J_i = W_i (Hadamard) [phi'(a_i) | ... | phi'(a_i)], phi' = cos. */
    for (int r = 0; r < R; ++r) {
      const double da = cos(a[r]);
      for (int c = 0; c < C; ++c) J[(size_t)r * C + c] = net->W[i][(size_t)r * C + c] * da;
    }
    /* Eq.(3), right to left: M <- J_i M. */
    for (int r = 0; r < R; ++r)
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int c = 0; c < C; ++c) s += J[(size_t)r * C + c] * M[c * 3 + j];
        Mn[r * 3 + j] = s;
      }
    for (int r = 0; r < R; ++r) hn[r] = sin(a[r]);
    double* t1 = h; h = hn; hn = t1;
    double* t2 = M; M = Mn; Mn = t2;
  }
  const int K = net->n_sine, C = net->cols[K];
  double out = net->b[K][0];
  for (int c = 0; c < C; ++c) out += net->W[K][c] * h[c];
  for (int j = 0; j < 3; ++j) {
    double s = 0.0;
    for (int c = 0; c < C; ++c) s += net->W[K][c] * M[c * 3 + j];
    grad[j] = s;
  }
  return out;
}

/* c(t) = rho (cos 2 pi t, sin 2 pi t, 0); rho = 0 is the static centre c = 0,
   whatever t holds. */
static void center_at(double rho, double t, double c[3]) {
  const double two_pi = 6.283185307179586476925286766559;
  c[0] = rho == 0.0 ? 0.0 : rho * cos(two_pi * t);
  c[1] = rho == 0.0 ? 0.0 : rho * sin(two_pi * t);
  c[2] = 0.0;
}

static void level_input(const orc_level* L, const double x[3], const double c[3], double t, double in[4]) {
  if (L->net.d_in == 4) {
    in[0] = x[0]; in[1] = x[1]; in[2] = x[2]; in[3] = t;
  } else if (L->follow_center) {
    in[0] = x[0] - c[0]; in[1] = x[1] - c[1]; in[2] = x[2] - c[2];
  } else {
    in[0] = x[0]; in[1] = x[1]; in[2] = x[2];
  }
}

/* f_j(x, t) = |x - c(t)| - r0 + a_j N_j(input) (without the first two terms when
   the base has no sphere). */
static double scene_value(const orc_level* L, const orc_base_desc* B, const double x[3], double t, double* ws) {
  double c[3], in[4];
  center_at(B->rho, t, c);
  const double dx = x[0] - c[0], dy = x[1] - c[1], dz = x[2] - c[2];
  const double base = B->sphere ? sqrt(dx * dx + dy * dy + dz * dz) - B->r0 : 0.0;
  if (L->amplitude == 0.0) return base;
  level_input(L, x, c, t, in);
  const size_t w = (size_t)(L->net.width > L->net.d_in ? L->net.width : L->net.d_in);
  return base + L->amplitude * net_value(&L->net, in, ws, ws + w);
}

/* f_j and grad_x f_j = (x - c)/|x - c| + a_j grad_x N_j. */
static double scene_value_grad(const orc_level* L, const orc_base_desc* B, const double x[3], double t,
                               double g[3], double* ws) {
  double c[3], in[4], gn[3] = {0.0, 0.0, 0.0};
  center_at(B->rho, t, c);
  const double d[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
  const double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  double nv = 0.0;
  if (L->amplitude != 0.0) {
    level_input(L, x, c, t, in);
    nv = net_value_grad(&L->net, in, gn, ws);
  }
  if (B->sphere) {
    for (int j = 0; j < 3; ++j) g[j] = (r > 0.0 ? d[j] / r : 0.0) + L->amplitude * gn[j];
    return r - B->r0 + L->amplitude * nv;
  }
  for (int j = 0; j < 3; ++j) g[j] = L->amplitude * gn[j];
  return L->amplitude * nv;
}

typedef struct {
  double step_scale, eps, far;
  int max_steps, final_level, normal_level;
  const int* iters; /* NULL: eps-terminated; else evaluations per traced level (fixed-iteration mode) */
} orc_trace_params;

/* One ray of multiscale sphere tracing (Algorithm 1).  Readings:
   - step: tau += s * d with d = f_j - delta_j, at every level, including the
     last small step (the loop evaluates, steps, then tests, as in Algorithm 1);
   - the last traced level uses delta = 0 (the ternary of Algorithm 1);
   - level switch when d <= eps; a miss when tau > far or when a level has used
     max_steps evaluations; a non-finite d is a miss flagged NONFINITE;
   - steps[j] counts the evaluations made at level j, on every exit (the one
     that ends the ray included), and stays 0 for levels never reached;
   - d < 0 (a start inside the band, which Algorithm 1 excludes) is flagged;
   - depth is the ray parameter tau of the point after the last step.
   Fixed-iteration mode (the paper's experiments fix the iteration counts): level
   j takes exactly iters[j] steps, with no eps exit; tau > far is still a miss;
   after the final traced level the ray is a hit when its last |d| <= eps, else
   a miss flagged BUDGET.
   Optional log: tau before each step, d, level (up to log_cap events). */
static int trace_one(const orc_level* lv, const orc_base_desc* B, const orc_trace_params* P,
                     const double o[3], const double v[3], double t, double* tau_out, uint8_t* steps,
                     double* ws, double* log_tau, double* log_d, int* log_level, int log_cap, int* n_log) {
  double tau = 0.0;
  int st = 0, nl = 0;
  for (int j = 0; j <= P->final_level; ++j) {
    const double delta = (j == P->final_level) ? 0.0 : lv[j].delta;
    int k = 0;
    for (;;) {
      const double p[3] = {o[0] + tau * v[0], o[1] + tau * v[1], o[2] + tau * v[2]};
      const double d = scene_value(&lv[j], B, p, t, ws) - delta;
      ++k;
      if (log_tau && nl < log_cap) {
        log_tau[nl] = tau;
        log_d[nl] = d;
        log_level[nl] = j;
        ++nl;
      }
      if (!isfinite(d)) {
        st |= ORC_ST_NONFINITE;
        if (steps) steps[j] = (uint8_t)k;
        goto miss;
      }
      if (d < 0.0) st |= ORC_ST_NEG_STEP;
      tau += P->step_scale * d;
      if (tau > P->far) {
        st |= ORC_ST_FAR;
        if (steps) steps[j] = (uint8_t)k;
        goto miss;
      }
      if (P->iters) {
        if (k < P->iters[j]) continue;
        if (j == P->final_level && fabs(d) > P->eps) {
          st |= ORC_ST_BUDGET;
          if (steps) steps[j] = (uint8_t)k;
          goto miss;
        }
        break;
      }
      if (d <= P->eps) break;
      if (k >= P->max_steps) {
        st |= ORC_ST_BUDGET;
        if (steps) steps[j] = (uint8_t)k;
        goto miss;
      }
    }
    if (steps) steps[j] = (uint8_t)k;
  }
  *tau_out = tau;
  if (n_log) *n_log = nl;
  return st | ORC_ST_HIT;
miss:
  *tau_out = INFINITY;
  if (n_log) *n_log = nl;
  return st;
}

static int levels_load(orc_level* lv, int m, const orc_level_desc* d) {
  for (int j = 0; j < m; ++j) {
    if (net_load(&lv[j].net, d[j].d_in, d[j].width, d[j].n_sine, d[j].params) != 0) {
      for (int q = 0; q < j; ++q) net_free(&lv[q].net);
      return -1;
    }
    lv[j].follow_center = d[j].follow_center;
    lv[j].amplitude = d[j].amplitude;
    lv[j].delta = d[j].delta;
  }
  return 0;
}

static void levels_free(orc_level* lv, int m) {
  for (int j = 0; j < m; ++j) net_free(&lv[j].net);
}

static size_t levels_ws(const orc_level* lv, int m) {
  size_t w = 0;
  for (int j = 0; j < m; ++j) {
    size_t s = net_ws_size(&lv[j].net);
    if (s > w) w = s;
  }
  return w;
}

static void set_threads(int threads) {
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#else
  (void)threads;
#endif
}

/* ---------------------------------------------------------------- exports */

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Raw network: N and grad N (first three inputs) at n points x[n][d_in].
   grad may be NULL (forward only). */
int orc_net_eval(int d_in, int width, int n_sine, const float* params, int64_t n, const double* x,
                 double* value, double* grad, int threads) {
  orc_net net;
  if (net_load(&net, d_in, width, n_sine, params) != 0) return -1;
  set_threads(threads);
  const size_t wsn = net_ws_size(&net);
  int err = 0;
#pragma omp parallel
  {
    double* ws = (double*)malloc(wsn * sizeof(double));
    if (!ws) {
#pragma omp atomic write
      err = -2;
    } else {
#pragma omp for schedule(dynamic, 16)
      for (int64_t i = 0; i < n; ++i) {
        if (grad) {
          value[i] = net_value_grad(&net, x + i * d_in, grad + 3 * i, ws);
        } else {
          const size_t w = (size_t)(width > d_in ? width : d_in);
          value[i] = net_value(&net, x + i * d_in, ws, ws + w);
        }
      }
      free(ws);
    }
  }
  net_free(&net);
  return err;
}

/* Scene function of one level: f and (optionally) grad_x f at x[n][3], times t[n] (or NULL). */
int orc_scene_eval(const orc_level_desc* level, const orc_base_desc* base, int64_t n, const double* x,
                   const double* t, double* value, double* grad, int threads) {
  orc_level L;
  if (levels_load(&L, 1, level) != 0) return -1;
  set_threads(threads);
  const size_t wsn = levels_ws(&L, 1);
  int err = 0;
#pragma omp parallel
  {
    double* ws = (double*)malloc(wsn * sizeof(double));
    if (!ws) {
#pragma omp atomic write
      err = -2;
    } else {
#pragma omp for schedule(dynamic, 16)
      for (int64_t i = 0; i < n; ++i) {
        const double ti = t ? t[i] : 0.0;
        if (grad)
          value[i] = scene_value_grad(&L, base, x + 3 * i, ti, grad + 3 * i, ws);
        else
          value[i] = scene_value(&L, base, x + 3 * i, ti, ws);
      }
      free(ws);
    }
  }
  levels_free(&L, 1);
  return err;
}

/* Multiscale sphere tracing of n rays (Algorithm 1) plus the unit normal of
   level normal_level at the end point of each hit (analytic normal; neural
   normal mapping when normal_level > final_level).
   o, v: [n][3] float32 (v unit); t: [n] or NULL.
   Outputs: depth[n] (+inf on a miss), hit[n], normal[n][3] (0 on a miss; may be
   NULL), steps[n][m] (evaluations per level; may be NULL), status[n] (may be NULL). */
int orc_trace_iters(int m, const orc_level_desc* levels, const orc_base_desc* base, double step_scale, double eps,
                    double far, int max_steps, const int* iters, int final_level, int normal_level, int64_t n,
                    const float* o, const float* v, const float* t, double* depth, uint8_t* hit, double* normal,
                    uint8_t* steps, uint8_t* status, int threads) {
  if (m < 1 || m > ORC_MAX_LEVELS || final_level < 0 || final_level >= m || normal_level < 0 ||
      normal_level >= m || max_steps < 1 || max_steps > 255)
    return -1;
  if (iters)
    for (int j = 0; j <= final_level; ++j)
      if (iters[j] < 1 || iters[j] > 255) return -1;
  orc_level lv[ORC_MAX_LEVELS];
  if (levels_load(lv, m, levels) != 0) return -1;
  orc_trace_params P = {step_scale, eps, far, max_steps, final_level, normal_level, iters};
  set_threads(threads);
  const size_t wsn = levels_ws(lv, m);
  int err = 0;
#pragma omp parallel
  {
    double* ws = (double*)malloc(wsn * sizeof(double));
    if (!ws) {
#pragma omp atomic write
      err = -2;
    } else {
#pragma omp for schedule(dynamic, 8)
      for (int64_t i = 0; i < n; ++i) {
        const double oi[3] = {o[3 * i], o[3 * i + 1], o[3 * i + 2]};
        const double vi[3] = {v[3 * i], v[3 * i + 1], v[3 * i + 2]};
        const double ti = t ? (double)t[i] : 0.0;
        uint8_t stp[ORC_MAX_LEVELS] = {0};
        double tau;
        const int st = trace_one(lv, base, &P, oi, vi, ti, &tau, stp, ws, NULL, NULL, NULL, 0, NULL);
        depth[i] = tau;
        hit[i] = (uint8_t)((st & ORC_ST_HIT) ? 1 : 0);
        if (status) status[i] = (uint8_t)st;
        if (steps)
          for (int j = 0; j < m; ++j) steps[i * m + j] = stp[j];
        if (normal) {
          double nrm[3] = {0.0, 0.0, 0.0};
          if (st & ORC_ST_HIT) {
            const double p[3] = {oi[0] + tau * vi[0], oi[1] + tau * vi[1], oi[2] + tau * vi[2]};
            double g[3];
            scene_value_grad(&lv[normal_level], base, p, ti, g, ws);
            const double len = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
            if (len > 0.0)
              for (int j = 0; j < 3; ++j) nrm[j] = g[j] / len;
          }
          for (int j = 0; j < 3; ++j) normal[3 * i + j] = nrm[j];
        }
      }
      free(ws);
    }
  }
  levels_free(lv, m);
  return err;
}

/* Eps-terminated multiscale sphere tracing (orc_trace_iters without iteration counts). */
int orc_trace(int m, const orc_level_desc* levels, const orc_base_desc* base, double step_scale, double eps,
              double far, int max_steps, int final_level, int normal_level, int64_t n, const float* o,
              const float* v, const float* t, double* depth, uint8_t* hit, double* normal, uint8_t* steps,
              uint8_t* status, int threads) {
  return orc_trace_iters(m, levels, base, step_scale, eps, far, max_steps, NULL, final_level, normal_level, n, o, v,
                         t, depth, hit, normal, steps, status, threads);
}

/* One ray with a log of every step: tau before the step, d, and the level.
   Returns the number of logged events (<= cap) and the status in *status. */
int orc_trace_log(int m, const orc_level_desc* levels, const orc_base_desc* base, double step_scale, double eps,
                  double far, int max_steps, int final_level, const float* o, const float* v, double t,
                  int cap, double* log_tau, double* log_d, int* log_level, double* tau_out, int* status) {
  if (m < 1 || m > ORC_MAX_LEVELS || final_level < 0 || final_level >= m) return -1;
  orc_level lv[ORC_MAX_LEVELS];
  if (levels_load(lv, m, levels) != 0) return -1;
  orc_trace_params P = {step_scale, eps, far, max_steps, final_level, final_level, NULL};
  double* ws = (double*)malloc(levels_ws(lv, m) * sizeof(double));
  if (!ws) {
    levels_free(lv, m);
    return -2;
  }
  const double oi[3] = {o[0], o[1], o[2]}, vi[3] = {v[0], v[1], v[2]};
  int nl = 0;
  *status = trace_one(lv, base, &P, oi, vi, t, tau_out, NULL, ws, log_tau, log_d, log_level, cap, &nl);
  free(ws);
  levels_free(lv, m);
  return nl;
}

/* Brute-force first zero crossing of f along o + tau v, tau in [0, far]: march
   with steps max(f / lip, h_min) (no root can lie within f / lip of a point when
   lip bounds |grad f|), then bisect the first sign change down to tol.
   Returns +inf when no crossing is found.  A check of the first-hit claim, not
   part of the method. */
int orc_first_root(const orc_level_desc* level, const orc_base_desc* base, int64_t n, const float* o,
                   const float* v, const float* t, double far, double lip, double h_min, double tol,
                   double* root, int threads) {
  orc_level L;
  if (levels_load(&L, 1, level) != 0) return -1;
  set_threads(threads);
  const size_t wsn = levels_ws(&L, 1);
  int err = 0;
#pragma omp parallel
  {
    double* ws = (double*)malloc(wsn * sizeof(double));
    if (!ws) {
#pragma omp atomic write
      err = -2;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (int64_t i = 0; i < n; ++i) {
        const double oi[3] = {o[3 * i], o[3 * i + 1], o[3 * i + 2]};
        const double vi[3] = {v[3 * i], v[3 * i + 1], v[3 * i + 2]};
        const double ti = t ? (double)t[i] : 0.0;
        double tau = 0.0;
        double p[3] = {oi[0], oi[1], oi[2]};
        double f = scene_value(&L, base, p, ti, ws);
        double res = INFINITY;
        if (f <= 0.0) {
          res = 0.0;
        } else {
          while (tau < far) {
            double step = f / lip;
            if (step < h_min) step = h_min;
            const double tn = tau + step;
            const double pn[3] = {oi[0] + tn * vi[0], oi[1] + tn * vi[1], oi[2] + tn * vi[2]};
            const double fn = scene_value(&L, base, pn, ti, ws);
            if (fn <= 0.0) {
              double lo = tau, hi = tn;
              while (hi - lo > tol) {
                const double mid = 0.5 * (lo + hi);
                const double pm[3] = {oi[0] + mid * vi[0], oi[1] + mid * vi[1], oi[2] + mid * vi[2]};
                if (scene_value(&L, base, pm, ti, ws) > 0.0)
                  lo = mid;
                else
                  hi = mid;
              }
              res = 0.5 * (lo + hi);
              break;
            }
            tau = tn;
            f = fn;
          }
        }
        root[i] = (res <= far) ? res : INFINITY;
      }
      free(ws);
    }
  }
  levels_free(&L, 1);
  return err;
}

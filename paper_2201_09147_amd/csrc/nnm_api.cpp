// nnm_api.cpp -- host side of libnnm's C ABI (include/nnm.h): validation,
// Lipschitz bounds, weight packing for the gfx950 kernels, and the launch
// sequence of multiscale sphere tracing.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "nnm.h"
#include "nnm_kernels.h"

using namespace nnm;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(NNM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

constexpr double kTwoPiD = 6.283185307179586476925286766559;

// Switches to a device for the lifetime of the guard.
struct DeviceGuard {
  int old = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&old) != hipSuccess) old = -1;
    if (old != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (old >= 0) (void)hipSetDevice(old);
  }
};

bool width_supported(int w) { return w == 32 || w == 64 || w == 128 || w == 256; }

// Shapes of the affine layers of a network: layer i is rows[i] x cols[i].
void layer_shape(int d_in, int width, int n_sine, int i, int* rows, int* cols) {
  *rows = (i == n_sine) ? 1 : width;
  *cols = (i == 0) ? d_in : width;
}

int64_t param_count(int d_in, int width, int n_sine) {
  int64_t total = 0;
  for (int i = 0; i <= n_sine; ++i) {
    int r, c;
    layer_shape(d_in, width, n_sine, i, &r, &c);
    total += (int64_t)r * c + r;
  }
  return total;
}

// Offsets of W_i and b_i in the flat parameter vector.
void layer_offsets(int d_in, int width, int n_sine, int i, int64_t* w_off, int64_t* b_off) {
  int64_t off = 0;
  for (int q = 0; q < i; ++q) {
    int r, c;
    layer_shape(d_in, width, n_sine, q, &r, &c);
    off += (int64_t)r * c + r;
  }
  int r, c;
  layer_shape(d_in, width, n_sine, i, &r, &c);
  *w_off = off;
  *b_off = off + (int64_t)r * c;
}

// Largest singular value of the rows x ncols block (leading columns of a
// rows x ld row-major matrix) by power iteration on W^T W in float64.
double spectral_norm(const float* W, int rows, int ld, int ncols) {
  std::vector<double> v(ncols), u(rows), w(ncols);
  for (int j = 0; j < ncols; ++j) v[j] = 1.0 + 0.01 * ((j * 37) % 11);
  double lam = 0.0;
  for (int it = 0; it < 1000; ++it) {
    double nv = 0.0;
    for (int j = 0; j < ncols; ++j) nv += v[j] * v[j];
    nv = std::sqrt(nv);
    if (nv == 0.0) return 0.0;
    for (int j = 0; j < ncols; ++j) v[j] /= nv;
    for (int r = 0; r < rows; ++r) {
      double s = 0.0;
      for (int j = 0; j < ncols; ++j) s += (double)W[(size_t)r * ld + j] * v[j];
      u[r] = s;
    }
    for (int j = 0; j < ncols; ++j) w[j] = 0.0;
    for (int r = 0; r < rows; ++r)
      for (int j = 0; j < ncols; ++j) w[j] += (double)W[(size_t)r * ld + j] * u[r];
    double nl = 0.0;
    for (int j = 0; j < ncols; ++j) nl += w[j] * v[j];
    v.swap(w);
    if (it > 10 && std::fabs(nl - lam) <= 1e-13 * std::fabs(nl)) {
      lam = nl;
      break;
    }
    lam = nl;
  }
  return std::sqrt(std::max(lam, 0.0));
}

double lipschitz_bound(const nnm_level_desc& L, int base_sphere) {
  double prod = 1.0;
  for (int i = 0; i <= L.n_sine; ++i) {
    int r, c;
    layer_shape(L.d_in, L.width, L.n_sine, i, &r, &c);
    int64_t wo, bo;
    layer_offsets(L.d_in, L.width, L.n_sine, i, &wo, &bo);
    prod *= spectral_norm(L.params + wo, r, c, i == 0 ? 3 : c);
  }
  return (base_sphere ? 1.0 : 0.0) + std::fabs((double)L.amplitude) * prod;
}

int validate_level(const nnm_level_desc& L, int j) {
  if (L.d_in != 3 && L.d_in != 4) return fail(NNM_E_UNSUPPORTED, "level %d: d_in %d (3 or 4 supported)", j, L.d_in);
  if (!width_supported(L.width))
    return fail(NNM_E_UNSUPPORTED, "level %d: width %d (32, 64, 128, 256 supported)", j, L.width);
  if (L.n_sine < 1 || L.n_sine > kMaxSine)
    return fail(NNM_E_UNSUPPORTED, "level %d: %d sine layers (1..%d supported)", j, L.n_sine, kMaxSine);
  if (!L.params) return fail(NNM_E_INVAL, "level %d: null params", j);
  if (!std::isfinite(L.amplitude)) return fail(NNM_E_NONFINITE, "level %d: non-finite amplitude", j);
  if (!std::isfinite(L.delta)) return fail(NNM_E_NONFINITE, "level %d: non-finite delta", j);
  const int64_t np = param_count(L.d_in, L.width, L.n_sine);
  for (int64_t k = 0; k < np; ++k)
    if (!std::isfinite(L.params[k])) return fail(NNM_E_NONFINITE, "level %d: non-finite parameter %lld", j, (long long)k);
  return NNM_OK;
}

uint16_t to_bf16_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}

uint16_t to_f16_rne(float x) {
  _Float16 h = (_Float16)x;  // round to nearest even
  uint16_t b;
  std::memcpy(&b, &h, 2);
  return b;
}

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct nnm_profiler {
  struct Rec {
    int kind, level, width, variant;
    hipEvent_t start, stop;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;  // reusable events
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void clear() {
    for (auto& r : recs) {
      pool.push_back(r.start);
      pool.push_back(r.stop);
    }
    recs.clear();
  }
  ~nnm_profiler() {
    clear();
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

namespace {
// Records an event pair around one launch when a profiler is attached.
struct ProfScope {
  nnm_profiler* p;
  nnm_profiler::Rec rec{};
  hipStream_t s;
  ProfScope(nnm_profiler* prof, int kind, int level, int width, int variant, hipStream_t st) : p(prof), s(st) {
    if (!p) return;
    rec.kind = kind;
    rec.level = level;
    rec.width = width;
    rec.variant = variant;
    rec.start = p->get();
    rec.stop = p->get();
    if (rec.start) (void)hipEventRecord(rec.start, s);
  }
  ~ProfScope() {
    if (!p || !rec.start || !rec.stop) return;
    (void)hipEventRecord(rec.stop, s);
    p->recs.push_back(rec);
  }
};
}  // namespace

struct nnm_stack {
  int device = 0;
  int precision = 0;
  int m = 0;
  DevBase base{};
  struct Level {
    int d_in, width, n_sine, follow_center;
    float amplitude, delta;
    DevLevel dev{};
    void* mem = nullptr;
    int resident[3] = {1, 1, 1};
    int ws_resident[2] = {1, 1};
  };
  std::vector<Level> levels;
};

extern "C" {

const char* nnm_last_error(void) { return g_err.c_str(); }

const char* nnm_version(void) { return "libnnm 0.1 (gfx950)"; }

void nnm_free(void* p) { std::free(p); }

int64_t nnm_param_count(int32_t d_in, int32_t width, int32_t n_sine) {
  if ((d_in != 3 && d_in != 4) || width < 1 || n_sine < 1 || n_sine > kMaxSine) return -1;
  return param_count(d_in, width, n_sine);
}

int nnm_level_lipschitz_bound(const nnm_level_desc* level, int base_sphere, double* bound) {
  if (!level || !bound) return fail(NNM_E_INVAL, "null argument");
  const int rc = validate_level(*level, 0);
  if (rc != NNM_OK) return rc;
  *bound = lipschitz_bound(*level, base_sphere);
  return NNM_OK;
}

int nnm_validate_stack(const nnm_stack_desc* d, int precision) {
  g_err.clear();
  if (!d) return fail(NNM_E_INVAL, "null stack descriptor");
  if (precision < NNM_PREC_FP32 || precision > NNM_PREC_FP16)
    return fail(NNM_E_UNSUPPORTED, "precision %d (0 fp32, 1 bf16, 2 fp16)", precision);
  if (d->n_levels < 1 || d->n_levels > kMaxLevels)
    return fail(NNM_E_INVAL, "n_levels %d (1..%d)", d->n_levels, kMaxLevels);
  if (!d->levels) return fail(NNM_E_INVAL, "null levels");
  if (!std::isfinite(d->r0) || !std::isfinite(d->rho) || !std::isfinite(d->lipschitz_max))
    return fail(NNM_E_NONFINITE, "non-finite base parameters");
  if (d->lipschitz_max < 0.f) return fail(NNM_E_INVAL, "negative lipschitz_max");
  for (int j = 0; j < d->n_levels; ++j) {
    const int rc = validate_level(d->levels[j], j);
    if (rc != NNM_OK) return rc;
  }
  // Nesting thresholds (Eq.(1)): delta_1 > delta_2 > ... > delta_{m-1} > 0.
  for (int j = 0; j + 1 < d->n_levels; ++j) {
    if (!(d->levels[j].delta > 0.f)) return fail(NNM_E_NESTING, "level %d: delta %g must be > 0", j, d->levels[j].delta);
    if (j > 0 && !(d->levels[j].delta < d->levels[j - 1].delta))
      return fail(NNM_E_NESTING, "level %d: delta %g not below delta %g of level %d", j, d->levels[j].delta,
                  d->levels[j - 1].delta, j - 1);
  }
  if (d->lipschitz_max > 0.f) {
    for (int j = 0; j < d->n_levels; ++j) {
      const double b = lipschitz_bound(d->levels[j], d->base_sphere);
      if (b > (double)d->lipschitz_max * (1.0 + 1e-6))
        return fail(NNM_E_LIPSCHITZ, "level %d: Lipschitz bound %.6f exceeds %.6f", j, b, (double)d->lipschitz_max);
    }
  }
  return NNM_OK;
}

static int pack_level(const nnm_level_desc& L, int precision, int device, nnm_stack::Level* out) {
  const int H = L.width, K = L.n_sine, MB = H / 32;
  // Host staging of every packed table.
  std::vector<float> a0(3 * MB * 64, 0.f);
  std::vector<float> bh((size_t)std::max(K - 1, 1) * H, 0.f);
  std::vector<float> wk(H, 0.f);
  const size_t elem = precision == NNM_PREC_FP32 ? 4 : 2;
  const size_t ah_stride = align256((size_t)H * H * elem);
  std::vector<uint8_t> ah((size_t)std::max(K - 1, 1) * ah_stride, 0);

  int64_t wo, bo;
  layer_offsets(L.d_in, H, K, 0, &wo, &bo);
  const float* W0 = L.params + wo;
  const float* b0 = L.params + bo;
  const int ncol0 = L.d_in + 1;  // augmented columns: inputs, then the bias
  for (int ks = 0; ks < 3; ++ks)
    for (int mb = 0; mb < MB; ++mb)
      for (int lane = 0; lane < 64; ++lane) {
        const int i = lane % 32, g = lane / 32, k = 2 * ks + g;
        const int row = 32 * mb + i;
        double v = 0.0;
        if (k < L.d_in)
          v = (double)W0[(size_t)row * L.d_in + k];
        else if (k == L.d_in)
          v = (double)b0[row];
        (void)ncol0;
        a0[a0_index(ks, mb, lane, MB)] = (float)(v / kTwoPiD);
      }
  // Largest input inf-norm X with |W_0 x + b_0| <= 63 revolutions in every
  // row (the tangent columns add a quarter revolution; the hardware sine is
  // accurate to 64): X = min over rows of (63 - |b_r|) / sum_k |W_0[r][k]| (in
  // revolutions, with a 1e-3 relative margin); -1 when a bias alone exceeds it.
  double l0_safe = 1e30;
  for (int row = 0; row < H; ++row) {
    double a = 0.0;
    for (int k = 0; k < L.d_in; ++k) a += std::fabs((double)W0[(size_t)row * L.d_in + k]);
    const double b = std::fabs((double)b0[row]) / kTwoPiD;
    a /= kTwoPiD;
    if (b >= 63.0) {
      l0_safe = -1.0;
      break;
    }
    if (a > 0.0) l0_safe = std::min(l0_safe, (63.0 - b) / a);
  }
  if (l0_safe > 0.0) l0_safe = std::min(l0_safe * (1.0 - 1e-3), 1e30);
  double hidden_arg = 0.0;  // bound of |hidden pre-activation| in revolutions
  for (int layer = 1; layer < K; ++layer) {
    layer_offsets(L.d_in, H, K, layer, &wo, &bo);
    const float* W = L.params + wo;
    const float* b = L.params + bo;
    for (int mb = 0; mb < MB; ++mb)
      for (int g = 0; g < 2; ++g)
        for (int r = 0; r < 16; ++r)
          bh[(size_t)(layer - 1) * H + acc_slot(mb, g, r)] = (float)((double)b[acc_row(mb, g, r)] / kTwoPiD);
    for (int row = 0; row < H; ++row) {
      double s = std::fabs((double)b[row]);
      for (int c = 0; c < H; ++c) s += std::fabs((double)W[(size_t)row * H + c]);
      hidden_arg = std::max(hidden_arg, s / kTwoPiD);
    }
    uint8_t* dst = ah.data() + (size_t)(layer - 1) * ah_stride;
    auto wscaled = [&](int row, int col) { return (float)((double)W[(size_t)row * H + col] / kTwoPiD); };
    if (precision == NNM_PREC_FP32) {
      float* A = (float*)dst;
      for (int q = 0; q < H / 8; ++q)
        for (int mb = 0; mb < MB; ++mb)
          for (int lane = 0; lane < 64; ++lane)
            for (int e = 0; e < 4; ++e) {
              const int i = lane % 32, g = lane / 32, ks = 4 * q + e;
              A[(((size_t)q * MB + mb) * 64 + lane) * 4 + e] = wscaled(32 * mb + i, kperm_2(ks, g));
            }
    } else {
      uint16_t* A = (uint16_t*)dst;
      for (int ks = 0; ks < 2 * MB; ++ks)
        for (int mb = 0; mb < MB; ++mb)
          for (int lane = 0; lane < 64; ++lane)
            for (int e = 0; e < 8; ++e) {
              const int i = lane % 32, g = lane / 32;
              const float w = wscaled(32 * mb + i, kperm_16(ks, g, e));
              A[(((size_t)ks * MB + mb) * 64 + lane) * 8 + e] =
                  precision == NNM_PREC_BF16 ? to_bf16_rne(w) : to_f16_rne(w);
            }
    }
  }
  layer_offsets(L.d_in, H, K, K, &wo, &bo);
  for (int mb = 0; mb < MB; ++mb)
    for (int g = 0; g < 2; ++g)
      for (int r = 0; r < 16; ++r) wk[acc_slot(mb, g, r)] = L.params[wo + acc_row(mb, g, r)];
  const float bk = L.params[bo];

  // Weight-stationary copy for width-256 nets with two hidden layers in
  // bf16/fp16: wave w of a workgroup holds rows [64 w, 64 w + 64), natural K order.
  const bool ws = (H == 256 && K == 3 && precision != NNM_PREC_FP32);
  std::vector<float> ws_a0, bh_plain, wk_plain;
  std::vector<uint16_t> ws_ah;
  if (ws) {
    ws_a0.assign(4 * 2 * 3 * 64, 0.f);
    for (int w = 0; w < 4; ++w)
      for (int rb = 0; rb < 2; ++rb)
        for (int ks = 0; ks < 3; ++ks)
          for (int lane = 0; lane < 64; ++lane) {
            const int row = 64 * w + 32 * rb + lane % 32, k = 2 * ks + lane / 32;
            double v = 0.0;
            if (k < L.d_in)
              v = (double)W0[(size_t)row * L.d_in + k];
            else if (k == L.d_in)
              v = (double)b0[row];
            ws_a0[((w * 2 + rb) * 3 + ks) * 64 + lane] = (float)(v / kTwoPiD);
          }
    ws_ah.assign((size_t)2 * 4 * 2 * 16 * 64 * 8, 0);
    bh_plain.assign(2 * 256, 0.f);
    for (int layer = 1; layer < K; ++layer) {
      int64_t wo2, bo2;
      layer_offsets(L.d_in, H, K, layer, &wo2, &bo2);
      const float* W = L.params + wo2;
      for (int row = 0; row < 256; ++row)
        bh_plain[(layer - 1) * 256 + row] = (float)((double)L.params[bo2 + row] / kTwoPiD);
      for (int w = 0; w < 4; ++w)
        for (int rb = 0; rb < 2; ++rb)
          for (int ks = 0; ks < 16; ++ks)
            for (int lane = 0; lane < 64; ++lane)
              for (int e = 0; e < 8; ++e) {
                const int row = 64 * w + 32 * rb + lane % 32, col = 16 * ks + 8 * (lane / 32) + e;
                const float v = (float)((double)W[(size_t)row * H + col] / kTwoPiD);
                ws_ah[(((((size_t)(layer - 1) * 4 + w) * 2 + rb) * 16 + ks) * 64 + lane) * 8 + e] =
                    precision == NNM_PREC_BF16 ? to_bf16_rne(v) : to_f16_rne(v);
              }
    }
    int64_t wok, bok;
    layer_offsets(L.d_in, H, K, K, &wok, &bok);
    wk_plain.assign(L.params + wok, L.params + wok + 256);
  }

  // One device allocation per level.
  const size_t off_a0 = 0;
  const size_t off_bh = off_a0 + align256(a0.size() * 4);
  const size_t off_wk = off_bh + align256(bh.size() * 4);
  const size_t off_ah = off_wk + align256(wk.size() * 4);
  const size_t off_ws_a0 = off_ah + align256(ah.size());
  const size_t off_ws_ah = off_ws_a0 + align256(ws_a0.size() * 4);
  const size_t off_bhp = off_ws_ah + align256(ws_ah.size() * 2);
  const size_t off_wkp = off_bhp + align256(bh_plain.size() * 4);
  const size_t total = off_wkp + align256(wk_plain.size() * 4);
  void* mem = nullptr;
  hipError_t e = hipMalloc(&mem, total);
  if (e != hipSuccess) return fail(NNM_E_NOMEM, "hipMalloc(%zu): %s", total, hipGetErrorString(e));
  char* base = (char*)mem;
  if ((e = hipMemcpy(base + off_a0, a0.data(), a0.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(base + off_bh, bh.data(), bh.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(base + off_wk, wk.data(), wk.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(base + off_ah, ah.data(), ah.size(), hipMemcpyHostToDevice)) != hipSuccess ||
      (ws && ((e = hipMemcpy(base + off_ws_a0, ws_a0.data(), ws_a0.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
              (e = hipMemcpy(base + off_ws_ah, ws_ah.data(), ws_ah.size() * 2, hipMemcpyHostToDevice)) != hipSuccess ||
              (e = hipMemcpy(base + off_bhp, bh_plain.data(), bh_plain.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
              (e = hipMemcpy(base + off_wkp, wk_plain.data(), wk_plain.size() * 4, hipMemcpyHostToDevice)) != hipSuccess))) {
    (void)hipFree(mem);
    return hip_fail(e, "uploading packed weights");
  }
  out->d_in = L.d_in;
  out->width = H;
  out->n_sine = K;
  out->follow_center = L.follow_center ? 1 : 0;
  out->amplitude = L.amplitude;
  out->delta = L.delta;
  out->mem = mem;
  DevLevel& D = out->dev;
  D.a0 = (const float*)(base + off_a0);
  D.bh = (const float*)(base + off_bh);
  D.wk = (const float*)(base + off_wk);
  D.ah = (const void*)(base + off_ah);
  D.ah_stride = (long long)ah_stride;
  D.bk = bk;
  D.amplitude = L.amplitude;
  D.delta = L.delta;
  D.d_in = L.d_in;
  D.width = H;
  D.n_sine = K;
  D.follow_center = out->follow_center;
  D.reduce_hidden = hidden_arg > 64.0 ? 1 : 0;
  D.l0_safe = (float)l0_safe;
  if (ws) {
    D.ws_a0 = (const float*)(base + off_ws_a0);
    D.ws_ah = (const void*)(base + off_ws_ah);
    D.bh_plain = (const float*)(base + off_bhp);
    D.wk_plain = (const float*)(base + off_wkp);
  }
  for (int kind = 0; kind < 3; ++kind) out->resident[kind] = resident_blocks(H, precision, kind, device);
  if (ws)
    for (int kind = 0; kind < 2; ++kind) out->ws_resident[kind] = ws_resident_blocks(precision, kind, device);
  return NNM_OK;
}

void free_siren_stack(nnm_stack* s) {
  if (!s) return;
  DeviceGuard guard(s->device);
  for (auto& L : s->levels)
    if (L.mem) (void)hipFree(L.mem);
  delete s;
}

int load_siren_stack(const nnm_stack_desc* d, int precision, int device, nnm_stack** out) {
  if (!out) return fail(NNM_E_INVAL, "null output handle");
  *out = nullptr;
  int rc = nnm_validate_stack(d, precision);
  if (rc != NNM_OK) return rc;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(NNM_E_DEVICE, "no HIP device");
  if (device < 0 || device >= ndev) return fail(NNM_E_INVAL, "device %d of %d", device, ndev);
  DeviceGuard guard(device);
  if (!guard.ok) return fail(NNM_E_DEVICE, "hipSetDevice(%d) failed", device);
  nnm_stack* s = new nnm_stack();
  s->device = device;
  s->precision = precision;
  s->m = d->n_levels;
  s->base.sphere = d->base_sphere ? 1 : 0;
  s->base.r0 = d->r0;
  s->base.rho = d->rho;
  s->levels.resize(d->n_levels);
  for (int j = 0; j < d->n_levels; ++j) {
    rc = pack_level(d->levels[j], precision, device, &s->levels[j]);
    if (rc != NNM_OK) {
      free_siren_stack(s);
      return rc;
    }
  }
  *out = s;
  return NNM_OK;
}

// A level reads the time when its network takes (x, t), or when its input or
// the base term follows the moving centre c(t).
static bool level_reads_time(const nnm_stack* s, int j) {
  const auto& L = s->levels[j];
  return L.d_in == 4 || (s->base.rho != 0.f && (s->base.sphere || L.follow_center));
}

int nnm_stack_levels(const nnm_stack* s) { return s ? s->m : -1; }
int nnm_stack_precision(const nnm_stack* s) { return s ? s->precision : -1; }

// Scratch of one trace_rays call: counters, two ping-pong queues, the order
// keys of the queue being written (by queue position), and the status carrier
// when the caller passes none.
struct TraceScratch {
  // counters: [0, 64) queue counts per level; then per level kOrderKeys key
  // totals and kOrderKeys reservation counters; then per level kSegments pop
  // counters kHeadStride ints apart
  static constexpr int n_fixed = 64 + kMaxLevels * 2 * kOrderKeys;
  static constexpr int n_cnt = n_fixed + kMaxLevels * kSegments * kHeadStride;
  size_t off_qa, off_qb, off_key, off_st, total;
  constexpr TraceScratch(int64_t n, bool status) : off_qa(0), off_qb(0), off_key(0), off_st(0), total(0) {
    off_qa = align256((size_t)n_cnt * 4);
    off_qb = off_qa + align256((size_t)n * 4);
    off_key = off_qb + align256((size_t)n * 4);
    off_st = off_key + align256((size_t)n);
    total = off_st + (status ? 0 : align256((size_t)n));
  }
};

static int trace_validate(const nnm_stack* s, const nnm_trace_params* p, int64_t n, const float* o, const float* v,
                          const float* t, float* depth, uint8_t* hit, float* normal) {
  if (!s || !p) return fail(NNM_E_INVAL, "null stack or params");
  if (n < 0) return fail(NNM_E_INVAL, "n = %lld < 0", (long long)n);
  if (n > (int64_t)INT_MAX - (1 << 24)) return fail(NNM_E_INVAL, "n = %lld too large", (long long)n);
  if (p->final_level < 0 || p->final_level >= s->m)
    return fail(NNM_E_INVAL, "final_level %d of %d levels", p->final_level, s->m);
  if (p->normal_level < 0 || p->normal_level >= s->m)
    return fail(NNM_E_INVAL, "normal_level %d of %d levels", p->normal_level, s->m);
  if (!(p->step_scale > 0.f && p->step_scale <= 1.f)) return fail(NNM_E_INVAL, "step_scale %g not in (0, 1]", p->step_scale);
  if (!(p->eps > 0.f) || !std::isfinite(p->eps)) return fail(NNM_E_INVAL, "eps %g", p->eps);
  if (!(p->far > 0.f) || !std::isfinite(p->far)) return fail(NNM_E_INVAL, "far %g", p->far);
  if (p->max_steps < 1 || p->max_steps > 255) return fail(NNM_E_INVAL, "max_steps %d not in 1..255", p->max_steps);
  if (p->mode != 0 && p->mode != 1) return fail(NNM_E_INVAL, "trace mode %d", p->mode);
  if (p->kernels != NNM_KERNELS_AUTO && p->kernels != NNM_KERNELS_STREAMING)
    return fail(NNM_E_INVAL, "kernel family %d", p->kernels);
  if (p->mode == 1)
    for (int j = 0; j <= p->final_level; ++j)
      if (p->iterations[j] < 1 || p->iterations[j] > 255)
        return fail(NNM_E_INVAL, "iterations[%d] = %d not in 1..255", j, p->iterations[j]);
  if (n == 0) return NNM_OK;
  if (!o || !v || !depth || !hit) return fail(NNM_E_INVAL, "null ray or output array");
  if (!t) {
    for (int j = 0; j <= p->final_level; ++j)
      if (level_reads_time(s, j)) return fail(NNM_E_INVAL, "null t, but level %d depends on the time", j);
    if (normal && level_reads_time(s, p->normal_level))
      return fail(NNM_E_INVAL, "null t, but normal level %d depends on the time", p->normal_level);
  }
  return NNM_OK;
}

// The launch sequence of one validated trace_rays call (n > 0) on the current
// device, with its scratch at wb (laid out by TraceScratch).  Every launch is
// a kernel (the counters are cleared by a fill kernel, not a memset).
static int trace_launch(const nnm_stack* s, const nnm_trace_params* p, int64_t n, const float* o, const float* v,
                        const float* t, float* depth, uint8_t* hit, float* normal, uint8_t* steps, uint8_t* status,
                        char* wb, hipStream_t st) {
  const TraceScratch sc(n, status != nullptr);
  const int L = p->final_level + 1;
  int* cnt = (int*)wb;
  int* qa = (int*)(wb + sc.off_qa);
  int* qb = (int*)(wb + sc.off_qb);
  uint8_t* key = (uint8_t*)(wb + sc.off_key);
  uint8_t* stat = status ? status : (uint8_t*)(wb + sc.off_st);
  int rc = NNM_OK;
  hipError_t e;
  if ((e = launch_zero_ints(cnt, TraceScratch::n_fixed + L * kSegments * kHeadStride, st)) != hipSuccess)
    rc = hip_fail(e, "zeroing counters");
  // Level j pops in_q and appends to out_q.  Between tracing levels (mode 0)
  // the appended queue is counting-sorted by decreasing evaluation count into
  // the other buffer, which the next level pops; otherwise the buffers swap.
  const int* in_q = nullptr;
  int* out_q = qa;
  int* spare = qb;
  for (int j = 0; j < L && rc == NNM_OK; ++j) {
    const auto& lv = s->levels[j];
    const bool is_final = (j == L - 1);
    const bool sort_next = !is_final && p->mode == 0;
    int* hist = cnt + 64 + j * 2 * kOrderKeys;
    TraceLevelArgs a{};
    a.L = lv.dev;
    a.B = s->base;
    a.o = o;
    a.v = v;
    a.t = t;
    a.depth = depth;
    a.hit = hit;
    a.normal = normal;
    a.steps = steps;
    a.status = stat;
    a.in_queue = in_q;
    a.in_count = j == 0 ? nullptr : cnt + (j - 1);
    a.in_heads = cnt + TraceScratch::n_fixed + j * kSegments * kHeadStride;
    a.out_queue = (!is_final || normal) ? out_q : nullptr;
    a.out_count = cnt + j;
    a.out_key = sort_next ? key : nullptr;
    a.out_hist = sort_next ? hist : nullptr;
    a.n = (int)n;
    a.level = j;
    a.m = s->m;
    a.is_final = is_final ? 1 : 0;
    a.max_steps = p->max_steps;
    a.step_scale = p->step_scale;
    a.eps = p->eps;
    a.far = p->far;
    a.fixed_iters = p->mode == 1 ? p->iterations[j] : 0;
    a.delta = is_final ? 0.f : lv.delta;
    const bool ws_kernel = lv.dev.ws_ah && p->kernels == NNM_KERNELS_AUTO;
    {
      ProfScope prof(p->profiler, 0, j, lv.width, ws_kernel ? 1 : 0, st);
      if (ws_kernel) {
        const long long want = ((long long)n + kWsRaysPerBlock - 1) / kWsRaysPerBlock;
        const int grid = (int)std::max(1LL, std::min(want, (long long)lv.ws_resident[0]));
        if ((e = launch_trace_ws(s->precision, a, grid, st)) != hipSuccess) rc = hip_fail(e, "trace level (ws)");
      } else {
        const long long want = ((long long)n + 127) / 128;
        const int grid = (int)std::max(1LL, std::min(want, (long long)lv.resident[0]));
        if ((e = launch_trace_level(lv.width, s->precision, a, grid, st)) != hipSuccess) rc = hip_fail(e, "trace level");
      }
    }
    if (rc != NNM_OK || is_final) break;
    if (sort_next) {
      QueueOrderArgs qo{};
      qo.in = out_q;
      qo.count = cnt + j;
      qo.key = key;
      qo.hist = hist;
      qo.fill = hist + kOrderKeys;
      qo.out = spare;
      const int grid = (int)std::max(1LL, std::min(256LL, ((long long)n + 4095) / 4096));
      ProfScope prof(p->profiler, 2, j, 0, 0, st);
      if ((e = launch_queue_order(qo, grid, st)) != hipSuccess) rc = hip_fail(e, "queue order");
      in_q = spare;  // out_q is free again
    } else {
      in_q = out_q;
      std::swap(out_q, spare);
    }
  }
  if (rc == NNM_OK && normal) {
    const auto& nl = s->levels[p->normal_level];
    NormalArgs a{};
    a.L = nl.dev;
    a.B = s->base;
    a.o = o;
    a.v = v;
    a.t = t;
    a.depth = depth;
    a.normal = normal;
    a.queue = out_q;
    a.count = cnt + (L - 1);
    a.n = (int)n;
    const bool ws_kernel = nl.dev.ws_ah && p->kernels == NNM_KERNELS_AUTO;
    ProfScope prof(p->profiler, 1, p->normal_level, nl.width, ws_kernel ? 1 : 0, st);
    if (ws_kernel) {
      const long long want = ((long long)n + kWsPointsPerBlock - 1) / kWsPointsPerBlock;
      const int grid = (int)std::max(1LL, std::min(want, (long long)nl.ws_resident[1]));
      if ((e = launch_normal_ws(s->precision, a, grid, st)) != hipSuccess) rc = hip_fail(e, "normal pass (ws)");
    } else {
      const long long want = ((long long)n + 31) / 32;
      const int grid = (int)std::max(1LL, std::min(want, (long long)nl.resident[1]));
      if ((e = launch_normal(nl.width, s->precision, a, grid, st)) != hipSuccess) rc = hip_fail(e, "normal pass");
    }
  }
  return rc;
}

// Scratch of trace_rays_noalloc: one static array per GPU, sized for the
// largest call it accepts (NNM_NOALLOC_MAX_RAYS rays, status carrier included).
// In host code `scratch` only names the symbol: its device address comes from
// hipGetSymbolAddress, once per device, and only that address is used.
constexpr size_t kNoAllocScratchBytes = TraceScratch(NNM_NOALLOC_MAX_RAYS, false).total;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device `dev` (resolved on the
// first call for that device).
static int noalloc_scratch(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(NNM_E_DEVICE, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return fail(NNM_E_DEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = (char*)g_scratch_ptr[dev];
  return NNM_OK;
}

int trace_rays(const nnm_stack* s, const nnm_trace_params* p, int64_t n, const float* o, const float* v,
               const float* t, float* depth, uint8_t* hit, float* normal, uint8_t* steps, uint8_t* status,
               void* stream) {
  g_err.clear();
  int rc = trace_validate(s, p, n, o, v, t, depth, hit, normal);
  if (rc != NNM_OK || n == 0) return rc;
  DeviceGuard guard(s->device);
  if (!guard.ok) return fail(NNM_E_DEVICE, "hipSetDevice(%d) failed", s->device);
  hipStream_t st = (hipStream_t)stream;
  const TraceScratch sc(n, status != nullptr);
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, sc.total, st);
  if (e != hipSuccess) return fail(NNM_E_NOMEM, "hipMallocAsync(%zu): %s", sc.total, hipGetErrorString(e));
  rc = trace_launch(s, p, n, o, v, t, depth, hit, normal, steps, status, (char*)ws, st);
  if ((e = hipFreeAsync(ws, st)) != hipSuccess && rc == NNM_OK) rc = hip_fail(e, "hipFreeAsync");
  return rc;
}

int trace_rays_noalloc(const nnm_stack* s, const nnm_trace_params* p, int64_t n, const float* o, const float* v,
                       const float* t, float* depth, uint8_t* hit, float* normal, uint8_t* steps, uint8_t* status,
                       void* stream) {
  g_err.clear();
  int rc = trace_validate(s, p, n, o, v, t, depth, hit, normal);
  if (rc != NNM_OK) return rc;
  if (n > NNM_NOALLOC_MAX_RAYS)
    return fail(NNM_E_INVAL, "n = %lld exceeds the %d rays of the static scratch", (long long)n, NNM_NOALLOC_MAX_RAYS);
  if (p->profiler) return fail(NNM_E_INVAL, "a profiler creates events; trace_rays_noalloc takes none");
  if (n == 0) return NNM_OK;
  DeviceGuard guard(s->device);
  if (!guard.ok) return fail(NNM_E_DEVICE, "hipSetDevice(%d) failed", s->device);
  char* wb = nullptr;
  if ((rc = noalloc_scratch(s->device, &wb)) != NNM_OK) return rc;
  return trace_launch(s, p, n, o, v, t, depth, hit, normal, steps, status, wb, (hipStream_t)stream);
}

static int points_common(const nnm_stack* s, int level, int64_t n, const float* x, const float* t, float* value,
                         float* grad, void* stream, int raw) {
  g_err.clear();
  if (!s) return fail(NNM_E_INVAL, "null stack");
  if (level < 0 || level >= s->m) return fail(NNM_E_INVAL, "level %d of %d", level, s->m);
  if (n < 0) return fail(NNM_E_INVAL, "n = %lld < 0", (long long)n);
  if (n > (int64_t)INT_MAX - (1 << 24)) return fail(NNM_E_INVAL, "n = %lld too large", (long long)n);
  if (n == 0) return NNM_OK;
  if (!x) return fail(NNM_E_INVAL, "null points");
  if (!value && !grad) return fail(NNM_E_INVAL, "no output requested");
  if (!t && level_reads_time(s, level)) return fail(NNM_E_INVAL, "null t, but level %d depends on the time", level);
  DeviceGuard guard(s->device);
  if (!guard.ok) return fail(NNM_E_DEVICE, "hipSetDevice(%d) failed", s->device);
  const auto& lv = s->levels[level];
  PointsArgs a{};
  a.L = lv.dev;
  a.B = s->base;
  a.x = x;
  a.t = t;
  a.value = value;
  a.grad = grad;
  a.n = (int)n;
  a.raw = raw;
  a.x_stride = 3;
  const long long want = ((long long)n + 31) / 32;
  const int grid = (int)std::max(1LL, std::min(want, (long long)lv.resident[2]));
  const hipError_t e = launch_points(lv.width, s->precision, a, grid, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "point evaluation");
  return NNM_OK;
}

int analytic_normal(const nnm_stack* s, int level, int64_t n, const float* x, const float* t, float* value,
                    float* grad, void* stream) {
  if (!grad && n > 0) return fail(NNM_E_INVAL, "null gradient output");
  return points_common(s, level, n, x, t, value, grad, stream, 0);
}

int nnm_net_eval(const nnm_stack* s, int level, int64_t n, const float* x, const float* t, float* value,
                 float* grad, void* stream) {
  return points_common(s, level, n, x, t, value, grad, stream, 1);
}

// Sampled maximum of |f_level_a - g| over n splitmix64 points of [lo, hi]^3,
// where g is level_b's scene function or, when ref != null, a reference SDF.
static int sup_abs_common(const nnm_stack* s, int level_a, int level_b, const nnm_ref_sdf* ref, int64_t n,
                          uint64_t seed, float lo, float hi, float* out_max, void* stream) {
  DeviceGuard guard(s->device);
  if (!guard.ok) return fail(NNM_E_DEVICE, "hipSetDevice(%d) failed", s->device);
  hipStream_t st = (hipStream_t)stream;
  // time-conditioned nets or a moving base: the time is sampled too
  const bool with_t = s->levels[level_a].d_in == 4 || (!ref && s->levels[level_b].d_in == 4) || s->base.rho != 0.f;
  const int chunk = (int)std::min<int64_t>(n, 1 << 22);
  const size_t off_x = 0, off_t = align256((size_t)chunk * 12), off_a = off_t + align256((size_t)chunk * 4),
               off_b = off_a + align256((size_t)chunk * 4);
  const size_t total = off_b + align256((size_t)chunk * 4);
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, total, st);
  if (e != hipSuccess) return fail(NNM_E_NOMEM, "hipMallocAsync(%zu): %s", total, hipGetErrorString(e));
  char* wb = (char*)ws;
  float* x = (float*)(wb + off_x);
  float* t = with_t ? (float*)(wb + off_t) : nullptr;
  float* fa = (float*)(wb + off_a);
  float* fb = (float*)(wb + off_b);
  int rc = NNM_OK;
  if ((e = launch_zero_ints((int*)out_max, 1, st)) != hipSuccess) rc = hip_fail(e, "zeroing the maximum");
  for (int64_t base = 0; base < n && rc == NNM_OK; base += chunk) {
    const int cnt = (int)std::min<int64_t>(chunk, n - base);
    if ((e = launch_box_points(seed, base, cnt, lo, hi, x, t, st)) != hipSuccess) {
      rc = hip_fail(e, "sampling points");
      break;
    }
    if ((rc = points_common(s, level_a, cnt, x, t, fa, nullptr, stream, 0)) != NNM_OK) break;
    if (ref) {
      if ((e = launch_ref_sdf(x, cnt, ref->kind, ref->a, ref->b, fb, st)) != hipSuccess) {
        rc = hip_fail(e, "reference SDF");
        break;
      }
    } else if ((rc = points_common(s, level_b, cnt, x, t, fb, nullptr, stream, 0)) != NNM_OK) {
      break;
    }
    if ((e = launch_absdiff_max(fa, fb, cnt, (unsigned int*)out_max, st)) != hipSuccess) rc = hip_fail(e, "max reduction");
  }
  if ((e = hipFreeAsync(ws, st)) != hipSuccess && rc == NNM_OK) rc = hip_fail(e, "hipFreeAsync");
  return rc;
}

int nnm_sup_abs_diff(const nnm_stack* s, int level_a, int level_b, int64_t n, uint64_t seed, float lo, float hi,
                     float* out_max, void* stream) {
  g_err.clear();
  if (!s || !out_max) return fail(NNM_E_INVAL, "null stack or output");
  if (level_a < 0 || level_a >= s->m || level_b < 0 || level_b >= s->m)
    return fail(NNM_E_INVAL, "levels %d, %d of %d", level_a, level_b, s->m);
  if (n < 1) return fail(NNM_E_INVAL, "n = %lld < 1", (long long)n);
  if (!(lo < hi) || !std::isfinite(lo) || !std::isfinite(hi)) return fail(NNM_E_INVAL, "box [%g, %g]", lo, hi);
  return sup_abs_common(s, level_a, level_b, nullptr, n, seed, lo, hi, out_max, stream);
}

int nnm_sup_abs_err(const nnm_stack* s, int level, const nnm_ref_sdf* ref, int64_t n, uint64_t seed, float lo,
                    float hi, float* out_max, void* stream) {
  g_err.clear();
  if (!s || !ref || !out_max) return fail(NNM_E_INVAL, "null stack, shape or output");
  if (level < 0 || level >= s->m) return fail(NNM_E_INVAL, "level %d of %d", level, s->m);
  if (n < 1) return fail(NNM_E_INVAL, "n = %lld < 1", (long long)n);
  if (!(lo < hi) || !std::isfinite(lo) || !std::isfinite(hi)) return fail(NNM_E_INVAL, "box [%g, %g]", lo, hi);
  if (ref->kind != NNM_REF_SPHERE && ref->kind != NNM_REF_TORUS) return fail(NNM_E_INVAL, "reference shape %d", ref->kind);
  if (!(ref->a > 0.f) || !std::isfinite(ref->a) || (ref->kind == NNM_REF_TORUS && (!(ref->b > 0.f) || !std::isfinite(ref->b))))
    return fail(NNM_E_INVAL, "reference radii %g, %g", ref->a, ref->b);
  return sup_abs_common(s, level, -1, ref, n, seed, lo, hi, out_max, stream);
}

int nnm_nesting_thresholds(int proposition, int32_t m, const double* sup, double margin, double* delta) {
  g_err.clear();
  if (!sup || !delta) return fail(NNM_E_INVAL, "null bounds or output");
  if (m < 2 || m > NNM_MAX_LEVELS) return fail(NNM_E_INVAL, "m = %d outside 2..%d", m, NNM_MAX_LEVELS);
  if (proposition != NNM_NEST_PROP1 && proposition != NNM_NEST_PROP2)
    return fail(NNM_E_INVAL, "proposition %d (1 or 2)", proposition);
  if (!(margin >= 0.0) || !std::isfinite(margin)) return fail(NNM_E_INVAL, "margin %g", margin);
  const int first = proposition == NNM_NEST_PROP1 ? 1 : 0;
  double eps[NNM_MAX_LEVELS] = {0.0};
  for (int i = first; i < m; ++i) {
    if (!(sup[i] >= 0.0) || !std::isfinite(sup[i])) return fail(NNM_E_INVAL, "bound %d = %g", i, sup[i]);
    eps[i] = sup[i] + margin;
  }
  if (proposition == NNM_NEST_PROP1) {
    // Proposition 1: |f_i - f_{i-1}| < eps_i gives delta_m = eps_m, delta_{i-1} = delta_i + eps_i.
    delta[m - 1] = eps[m - 1];
    for (int i = m - 1; i >= 1; --i) delta[i - 1] = delta[i] + eps[i];
  } else {
    // Proposition 2: |f - f_i| < eps_i gives delta_m = eps_m + eps_{m-1},
    // delta_{i-1} = delta_i + eps_i + eps_{i-1}.
    delta[m - 1] = eps[m - 1] + eps[m - 2];
    for (int i = m - 1; i >= 1; --i) delta[i - 1] = delta[i] + eps[i] + eps[i - 1];
  }
  return NNM_OK;
}

int neural_normal_map(const nnm_stack* s, int level, int64_t n, const float* x, const float* t, float* normal,
                      void* stream) {
  g_err.clear();
  if (!s) return fail(NNM_E_INVAL, "null stack");
  if (level < 0 || level >= s->m) return fail(NNM_E_INVAL, "level %d of %d", level, s->m);
  if (n < 0) return fail(NNM_E_INVAL, "n = %lld < 0", (long long)n);
  if (n > (int64_t)INT_MAX - (1 << 24)) return fail(NNM_E_INVAL, "n = %lld too large", (long long)n);
  if (n == 0) return NNM_OK;
  if (!x || !normal) return fail(NNM_E_INVAL, "null points or normals");
  if (!t && level_reads_time(s, level)) return fail(NNM_E_INVAL, "null t, but level %d depends on the time", level);
  DeviceGuard guard(s->device);
  if (!guard.ok) return fail(NNM_E_DEVICE, "hipSetDevice(%d) failed", s->device);
  const auto& lv = s->levels[level];
  NormalArgs a{};
  a.L = lv.dev;
  a.B = s->base;
  a.t = t;
  a.normal = normal;
  a.n = (int)n;
  a.x = x;
  hipError_t e;
  if (lv.dev.ws_ah) {
    const long long want = (n + kWsPointsPerBlock - 1) / kWsPointsPerBlock;
    const int grid = (int)std::max(1LL, std::min(want, (long long)lv.ws_resident[1]));
    e = launch_normal_ws(s->precision, a, grid, (hipStream_t)stream);
  } else {
    const long long want = (n + 31) / 32;
    const int grid = (int)std::max(1LL, std::min(want, (long long)lv.resident[1]));
    e = launch_normal(lv.width, s->precision, a, grid, (hipStream_t)stream);
  }
  if (e != hipSuccess) return hip_fail(e, "normal mapping");
  return NNM_OK;
}

int nnm_grid_values(const nnm_stack* s, int level, int32_t res, float lo, float hi, float t, float* values,
                    void* stream) {
  g_err.clear();
  if (!s || !values) return fail(NNM_E_INVAL, "null stack or output");
  if (level < 0 || level >= s->m) return fail(NNM_E_INVAL, "level %d of %d", level, s->m);
  if (res < 2 || res > NNM_MESH_MAX_RES) return fail(NNM_E_INVAL, "res = %d outside [2, %d]", res, NNM_MESH_MAX_RES);
  if (!(lo < hi) || !std::isfinite(lo) || !std::isfinite(hi)) return fail(NNM_E_INVAL, "box [%g, %g]", lo, hi);
  if (!std::isfinite(t)) return fail(NNM_E_INVAL, "time %g", t);
  DeviceGuard guard(s->device);
  if (!guard.ok) return fail(NNM_E_DEVICE, "hipSetDevice(%d) failed", s->device);
  const auto& lv = s->levels[level];
  GridArgs a{};
  a.L = lv.dev;
  a.B = s->base;
  a.res = res;
  a.n = res * res * res;
  a.lo = lo;
  a.hi = hi;
  a.t = t;
  a.values = values;
  const hipError_t e = launch_grid_values(lv.width, s->precision, a, s->device, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "grid values");
  return NNM_OK;
}

int nnm_mesh_extract(const float* values, int32_t res, float lo, float hi, float iso, int64_t max_verts,
                     int64_t max_tris, float* verts, int32_t* tris, int64_t* counts, void* stream) {
  g_err.clear();
  if (!values || !counts) return fail(NNM_E_INVAL, "null values or counts");
  if (res < 2 || res > NNM_MESH_MAX_RES) return fail(NNM_E_INVAL, "res = %d outside [2, %d]", res, NNM_MESH_MAX_RES);
  if (!(lo < hi) || !std::isfinite(lo) || !std::isfinite(hi)) return fail(NNM_E_INVAL, "box [%g, %g]", lo, hi);
  if (!std::isfinite(iso)) return fail(NNM_E_INVAL, "iso %g", iso);
  if (max_verts < 0 || max_tris < 0) return fail(NNM_E_INVAL, "negative capacity");
  if ((max_verts > 0 && !verts) || (max_tris > 0 && !tris)) return fail(NNM_E_INVAL, "null output array");
  hipStream_t st = (hipStream_t)stream;
  MeshArgs a{};
  a.values = values;
  a.res = res;
  a.n_nodes = res * res * res;
  a.n_blocks = mesh_blocks(res);
  a.n_groups = (a.n_blocks + 1023) / 1024;
  a.lo = lo;
  a.hi = hi;
  a.iso = iso;
  a.verts = verts;
  a.tris = tris;
  a.max_v = max_verts;
  a.max_t = max_tris;
  a.counts = (long long*)counts;
  const size_t off_bt = align256((size_t)a.n_blocks * 4), off_gv = off_bt + align256((size_t)a.n_blocks * 4),
               off_gt = off_gv + align256((size_t)a.n_groups * 4), off_vo = off_gt + align256((size_t)a.n_groups * 4),
               off_fl = off_vo + align256((size_t)a.n_nodes * 4), total = off_fl + align256((size_t)a.n_nodes);
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, total, st);
  if (e != hipSuccess) return fail(NNM_E_NOMEM, "hipMallocAsync(%zu): %s", total, hipGetErrorString(e));
  char* wb = (char*)ws;
  a.bsum_v = (int*)wb;
  a.bsum_t = (int*)(wb + off_bt);
  a.gsum_v = (int*)(wb + off_gv);
  a.gsum_t = (int*)(wb + off_gt);
  a.vert_off = (int*)(wb + off_vo);
  a.mask = (uint8_t*)(wb + off_fl);
  int rc = NNM_OK;
  if ((e = launch_marching_tets(a, st)) != hipSuccess) rc = hip_fail(e, "marching tetrahedra");
  if ((e = hipFreeAsync(ws, st)) != hipSuccess && rc == NNM_OK) rc = hip_fail(e, "hipFreeAsync");
  return rc;
}

int nnm_profiler_create(nnm_profiler** out) {
  if (!out) return fail(NNM_E_INVAL, "null output handle");
  *out = new nnm_profiler();
  return NNM_OK;
}

void nnm_profiler_free(nnm_profiler* prof) { delete prof; }

int nnm_profiler_reset(nnm_profiler* prof) {
  if (!prof) return fail(NNM_E_INVAL, "null profiler");
  prof->clear();
  return NNM_OK;
}

int nnm_profiler_report(nnm_profiler* prof, nnm_profile_report* out) {
  if (!prof || !out) return fail(NNM_E_INVAL, "null argument");
  std::memset(out, 0, sizeof(*out));
  for (auto& r : prof->recs) {
    hipError_t e = hipEventSynchronize(r.stop);
    if (e != hipSuccess) return hip_fail(e, "profiler event");
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, r.start, r.stop);
    if (e != hipSuccess) return hip_fail(e, "profiler elapsed time");
    int slot = -1;
    for (int i = 0; i < out->n_entries; ++i)
      if (out->kind[i] == r.kind && out->level[i] == r.level && out->variant[i] == r.variant) slot = i;
    if (slot < 0) {
      if (out->n_entries >= NNM_PROF_MAX) continue;
      slot = out->n_entries++;
      out->kind[slot] = r.kind;
      out->level[slot] = r.level;
      out->width[slot] = r.width;
      out->variant[slot] = r.variant;
    }
    out->launches[slot] += 1;
    out->total_ms[slot] += ms;
  }
  return NNM_OK;
}

int nnm_sync(void* stream) {
  const hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  const hipError_t e2 = hipGetLastError();
  if (e2 != hipSuccess) return hip_fail(e2, "pending device error");
  return NNM_OK;
}

int nnm_write_net_file(const char* path, int32_t d_in, int32_t width, int32_t n_sine, const float* params,
                       int64_t n_params) {
  g_err.clear();
  if (!path || !params) return fail(NNM_E_INVAL, "null path or parameters");
  if ((d_in != 3 && d_in != 4) || width < 1 || width > 4096 || n_sine < 1 || n_sine > kMaxSine)
    return fail(NNM_E_INVAL, "shape d_in %d width %d n_sine %d", d_in, width, n_sine);
  if (n_params != param_count(d_in, width, n_sine))
    return fail(NNM_E_INVAL, "%lld parameters, expected %lld", (long long)n_params,
                (long long)param_count(d_in, width, n_sine));
  const std::string tmp = std::string(path) + ".tmp";
  FILE* fh = std::fopen(tmp.c_str(), "wb");
  if (!fh) return fail(NNM_E_IO, "cannot open %s", tmp.c_str());
  const uint32_t hdr[7] = {1u, (uint32_t)d_in, (uint32_t)width, (uint32_t)n_sine, 0u, 0u, 0u};
  bool ok = std::fwrite("NNMW", 1, 4, fh) == 4 && std::fwrite(hdr, 4, 7, fh) == 7 &&
            std::fwrite(params, 4, (size_t)n_params, fh) == (size_t)n_params;
  ok = (std::fclose(fh) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return fail(NNM_E_IO, "cannot write %s", path);
  }
  return NNM_OK;
}

int nnm_read_net_file(const char* path, int32_t* d_in, int32_t* width, int32_t* n_sine, float** params_out,
                      int64_t* n_params) {
  g_err.clear();
  if (!path || !d_in || !width || !n_sine || !params_out || !n_params) return fail(NNM_E_INVAL, "null argument");
  *params_out = nullptr;
  FILE* fh = std::fopen(path, "rb");
  if (!fh) return fail(NNM_E_IO, "cannot open %s", path);
  uint32_t hdr[8];
  char magic[4];
  if (std::fread(magic, 1, 4, fh) != 4 || std::fread(hdr, 4, 7, fh) != 7) {
    std::fclose(fh);
    return fail(NNM_E_FORMAT, "%s: short header", path);
  }
  if (std::memcmp(magic, "NNMW", 4) != 0) {
    std::fclose(fh);
    return fail(NNM_E_FORMAT, "%s: bad magic", path);
  }
  if (hdr[0] != 1) {
    std::fclose(fh);
    return fail(NNM_E_FORMAT, "%s: version %u", path, hdr[0]);
  }
  const int di = (int)hdr[1], w = (int)hdr[2], ns = (int)hdr[3];
  if ((di != 3 && di != 4) || w < 1 || w > 4096 || ns < 1 || ns > kMaxSine) {
    std::fclose(fh);
    return fail(NNM_E_FORMAT, "%s: shape d_in %d width %d n_sine %d", path, di, w, ns);
  }
  const int64_t np = param_count(di, w, ns);
  float* buf = (float*)std::malloc((size_t)np * 4);
  if (!buf) {
    std::fclose(fh);
    return fail(NNM_E_NOMEM, "malloc");
  }
  const size_t got = std::fread(buf, 4, (size_t)np, fh);
  char extra;
  const bool trailing = std::fread(&extra, 1, 1, fh) == 1;
  std::fclose(fh);
  if (got != (size_t)np || trailing) {
    std::free(buf);
    return fail(NNM_E_FORMAT, "%s: %zu parameters, expected %lld%s", path, got, (long long)np,
                trailing ? " (trailing bytes)" : "");
  }
  *d_in = di;
  *width = w;
  *n_sine = ns;
  *params_out = buf;
  *n_params = np;
  return NNM_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ fitting

namespace {

bool shape_ok(const nnm_net_shape* sh) {
  return sh && (sh->d_in == 3 || sh->d_in == 4) && width_supported(sh->width) && sh->n_sine >= 1 &&
         sh->n_sine <= kMaxSine;
}

// Layout of the fitting workspace for n points.
struct FitLayout {
  long long Kc = 0;
  int nwaves = 0;
  size_t off_a0, off_bh, off_wk, off_bk, off_ah, off_aht, off_w0t;
  size_t off_abar, off_x, off_adj, off_mask, off_wvec, off_loss, off_part;
  long long chunk_w = 0;
  int nchunk_w = 0;
  size_t total;
};

FitLayout fit_layout(const nnm_net_shape& sh, int64_t n, int grid) {
  FitLayout L;
  const size_t H = sh.width, K = sh.n_sine, MB = H / 32;
  L.Kc = 32LL * ((n + 7) / 8);
  if (L.Kc == 0) L.Kc = 32;
  L.nwaves = grid * (kBlockThreads / 64);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += align256(bytes);
    return at;
  };
  L.off_a0 = take(3 * MB * 64 * 4);
  L.off_bh = take(std::max<size_t>(K - 1, 1) * H * 4);
  L.off_wk = take(H * 4);
  L.off_bk = take(4);
  L.off_ah = take(std::max<size_t>(K - 1, 1) * H * H * 4);
  L.off_aht = take(std::max<size_t>(K - 1, 1) * H * H * 4);
  L.off_w0t = take(H * 16);
  L.off_abar = take(K * H * (size_t)L.Kc * 4);
  L.off_x = take(K * H * (size_t)L.Kc * 4);
  L.off_adj = take((size_t)L.Kc * 4);
  // mask and the d_in column-weight vectors are one contiguous [1 + d_in][Kc] block
  L.off_mask = take((size_t)(1 + sh.d_in) * L.Kc * 4);
  L.off_wvec = L.off_mask + (size_t)L.Kc * 4;
  L.off_loss = take((size_t)L.nwaves * 16 + 16);
  // partial sums of the weight-gradient reductions (used one after another)
  L.chunk_w = std::max(64LL, ((L.Kc + 255) / 256 + 15) & ~15LL);  // whole column batches
  L.nchunk_w = (int)((L.Kc + L.chunk_w - 1) / L.chunk_w);
  const size_t col_part = (size_t)colreduce_blocks(L.Kc, (int)H) * 5 * H;
  L.off_part = take(std::max({col_part, (size_t)L.nchunk_w * H * H, (size_t)kSumBlocks}) * 4);
  L.total = o;
  return L;
}

// Packs `params` and runs the forward/adjoint and reverse launches plus the
// gradient products.  mode 0: loss (batch), mode 1: upstream adjoints.
int fit_backward_impl(const nnm_net_shape& sh, const float* params, int device, int grid, char* ws,
                      const FitLayout& FL, int mode, int64_t n, int64_t n_surf, const float* x0, const float* x1,
                      const float* surf_n, const float* unif_sdf, const float* dvalue, const float* dgrad,
                      float* loss4, float* dparams, float* dx, hipStream_t st) {
  const int H = sh.width, K = sh.n_sine;
  FitPackArgs pk{};
  pk.params = params;
  pk.d_in = sh.d_in;
  pk.width = H;
  pk.n_sine = K;
  for (int i = 0; i <= K; ++i) {
    int64_t wo, bo;
    layer_offsets(sh.d_in, H, K, i, &wo, &bo);
    pk.w_off[i] = wo;
    pk.b_off[i] = bo;
  }
  pk.a0 = (float*)(ws + FL.off_a0);
  pk.bh = (float*)(ws + FL.off_bh);
  pk.wk = (float*)(ws + FL.off_wk);
  pk.bk = (float*)(ws + FL.off_bk);
  pk.ah = (float*)(ws + FL.off_ah);
  pk.aht = (float*)(ws + FL.off_aht);
  pk.w0t = (float4*)(ws + FL.off_w0t);
  hipError_t e;
  if ((e = launch_fit_pack(pk, st)) != hipSuccess) return hip_fail(e, "fit pack");
  FitVecArgs va{};
  va.Kc = FL.Kc;
  va.n = (int)n;
  va.n_surf = (int)n_surf;
  va.mode = mode;
  va.d_in = sh.d_in;
  va.x0 = x0;
  va.x1 = x1;
  va.mask = (float*)(ws + FL.off_mask);
  va.wvec = (float*)(ws + FL.off_wvec);
  if ((e = launch_fit_vectors(va, st)) != hipSuccess) return hip_fail(e, "fit vectors");
  FitArgs a{};
  DevLevel& D = a.L;
  D.a0 = pk.a0;
  D.bh = pk.bh;
  D.wk = pk.wk;
  D.ah = pk.ah;
  D.ah_stride = (long long)H * H * 4;
  D.bk = 0.f;
  D.bk_dev = pk.bk;
  D.amplitude = 1.f;
  D.d_in = sh.d_in;
  D.width = H;
  D.n_sine = K;
  D.reduce_hidden = 1;
  D.l0_safe = -1.f;
  a.aht = pk.aht;
  a.w0t = pk.w0t;
  a.n = (int)n;
  a.n_surf = (int)n_surf;
  a.mode = mode;
  a.x0 = x0;
  a.x1 = x1;
  a.surf_n = surf_n;
  a.unif_sdf = unif_sdf;
  a.dvalue = dvalue;
  a.dgrad = dgrad;
  a.inv_ns = n_surf > 0 ? 1.f / (float)n_surf : 0.f;
  a.inv_nu = (n - n_surf) > 0 ? 1.f / (float)(n - n_surf) : 0.f;
  a.ws_abar = (float*)(ws + FL.off_abar);
  a.ws_x = (float*)(ws + FL.off_x);
  a.adj = (float*)(ws + FL.off_adj);
  a.loss_part = (float*)(ws + FL.off_loss);
  a.dx = dx;
  a.Kc = FL.Kc;
  if ((e = launch_fit_fb(a, grid, st)) != hipSuccess) return hip_fail(e, "fit forward/backward");
  if (loss4 && mode == 0)
    if ((e = launch_fit_loss_reduce(a.loss_part, FL.nwaves, a.inv_ns, a.inv_nu, loss4, st)) != hipSuccess)
      return hip_fail(e, "loss reduce");
  // Gradient products over the workspace slabs ([column][neuron]), each column
  // read once, partial sums over column chunks added in a fixed order.
  const int d_in = sh.d_in;
  const float* abar = a.ws_abar;
  const float* X = a.ws_x;
  const size_t LS = (size_t)H * FL.Kc;  // floats per layer slab
  float* part = (float*)(ws + FL.off_part);
  for (int i = 1; i < K; ++i) {
    // W_i-bar[out][in] = sum_col abar_i[col][out] X_i[col][in], X_i = inputs of layer i
    if ((e = launch_wgrad(H, abar + i * LS, X + (i - 1) * LS, FL.Kc, (int)FL.chunk_w, part, dparams + pk.w_off[i],
                          st)) != hipSuccess)
      return hip_fail(e, "hidden weight gradient");
  }
  // layer 0: b_0-bar (primal mask) and W_0-bar[:, j] (column weights w_j); the
  // mask and the w_j are contiguous vectors of length Kc in the workspace.
  // Point p owns columns 4p (primal) .. 4p+3 (tangents), so a reduction
  // weighted by the primal mask alone reads every fourth column.
  {
    ColDst dst{};
    dst.ptr[0] = dparams + pk.b_off[0];
    dst.stride[0] = 1;
    for (int j = 0; j < d_in; ++j) {
      dst.ptr[1 + j] = dparams + pk.w_off[0] + j;
      dst.stride[1 + j] = d_in;
    }
    if ((e = launch_colreduce(abar, H, FL.Kc, va.mask, 1 + d_in, 1, part, dst, st)) != hipSuccess)
      return hip_fail(e, "first-layer gradient");
  }
  for (int i = 1; i < K; ++i) {
    ColDst dst{};
    dst.ptr[0] = dparams + pk.b_off[i];
    dst.stride[0] = 1;
    if ((e = launch_colreduce(abar + i * LS, H, FL.Kc, va.mask, 1, 4, part, dst, st)) != hipSuccess)
      return hip_fail(e, "bias gradient");
  }
  {
    ColDst dst{};
    dst.ptr[0] = dparams + pk.w_off[K];
    dst.stride[0] = 1;
    if ((e = launch_colreduce(X + (K - 1) * LS, H, FL.Kc, a.adj, 1, 1, part, dst, st)) != hipSuccess)
      return hip_fail(e, "output-layer gradient");
  }
  if ((e = launch_masked_sum(a.adj, va.mask, FL.Kc, 4, part, dparams + pk.b_off[K], st)) != hipSuccess)
    return hip_fail(e, "output-bias gradient");
  return NNM_OK;
}

int current_device(int* dev) {
  return hipGetDevice(dev) == hipSuccess ? NNM_OK : fail(NNM_E_DEVICE, "hipGetDevice failed");
}

}  // namespace

struct nnm_fit {
  int device = 0;
  nnm_net_shape shape{};
  int64_t n_params = 0;
  int64_t max_points = 0;
  int grid = 1;
  float* state = nullptr;  // params | m | v | grad
  char* ws = nullptr;
  FitLayout layout{};
  int64_t step = 0;
};

extern "C" {

int64_t siren_workspace_bytes(const nnm_net_shape* shape, int64_t n) {
  if (!shape_ok(shape) || n < 0) return -1;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  return (int64_t)fit_layout(*shape, n, fit_fb_grid(shape->width, dev)).total;
}

int siren_forward_tangent(const nnm_net_shape* shape, const float* params, int64_t n, const float* x, float* value,
                          float* grad, void* stream) {
  g_err.clear();
  if (!shape_ok(shape)) return fail(NNM_E_UNSUPPORTED, "unsupported network shape");
  if (n < 0 || n > (int64_t)INT_MAX / 8) return fail(NNM_E_INVAL, "n = %lld", (long long)n);
  if (n == 0) return NNM_OK;
  if (!params || !x || (!value && !grad)) return fail(NNM_E_INVAL, "null argument");
  int dev;
  if (current_device(&dev) != NNM_OK) return NNM_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  // Pack into a small stream-ordered scratch, then evaluate with the points kernel.
  const FitLayout FL = fit_layout(*shape, 0, 1);
  const size_t pack_bytes = FL.off_abar;
  void* ws = nullptr;
  hipError_t e = hipMallocAsync(&ws, pack_bytes, st);
  if (e != hipSuccess) return fail(NNM_E_NOMEM, "hipMallocAsync(%zu)", pack_bytes);
  char* w = (char*)ws;
  FitPackArgs pk{};
  pk.params = params;
  pk.d_in = shape->d_in;
  pk.width = shape->width;
  pk.n_sine = shape->n_sine;
  for (int i = 0; i <= shape->n_sine; ++i) {
    int64_t wo, bo;
    layer_offsets(shape->d_in, shape->width, shape->n_sine, i, &wo, &bo);
    pk.w_off[i] = wo;
    pk.b_off[i] = bo;
  }
  pk.a0 = (float*)(w + FL.off_a0);
  pk.bh = (float*)(w + FL.off_bh);
  pk.wk = (float*)(w + FL.off_wk);
  pk.bk = (float*)(w + FL.off_bk);
  pk.ah = (float*)(w + FL.off_ah);
  pk.aht = (float*)(w + FL.off_aht);
  pk.w0t = (float4*)(w + FL.off_w0t);
  int rc = NNM_OK;
  if ((e = launch_fit_pack(pk, st)) != hipSuccess) rc = hip_fail(e, "pack");
  if (rc == NNM_OK) {
    PointsArgs a{};
    DevLevel& D = a.L;
    D.a0 = pk.a0;
    D.bh = pk.bh;
    D.wk = pk.wk;
    D.ah = pk.ah;
    D.ah_stride = (long long)shape->width * shape->width * 4;
    D.bk_dev = pk.bk;
    D.amplitude = 1.f;
    D.d_in = shape->d_in;
    D.width = shape->width;
    D.n_sine = shape->n_sine;
    D.reduce_hidden = 1;
    D.l0_safe = -1.f;
    a.x = x;
    a.t = nullptr;
    a.value = value;
    a.grad = grad;
    a.n = (int)n;
    a.raw = 1;
    a.x_stride = shape->d_in;
    const int grid = (int)std::max(1LL, std::min(((long long)n + 31) / 32,
                                                 (long long)resident_blocks(shape->width, NNM_PREC_FP32, 2, dev)));
    if ((e = launch_points(shape->width, NNM_PREC_FP32, a, grid, st)) != hipSuccess) rc = hip_fail(e, "forward");
  }
  if ((e = hipFreeAsync(ws, st)) != hipSuccess && rc == NNM_OK) rc = hip_fail(e, "hipFreeAsync");
  return rc;
}

int siren_backward(const nnm_net_shape* shape, const float* params, int64_t n, const float* x, const float* dvalue,
                   const float* dgrad, float* dparams, float* dx, void* workspace, int64_t workspace_bytes,
                   void* stream) {
  g_err.clear();
  if (!shape_ok(shape)) return fail(NNM_E_UNSUPPORTED, "unsupported network shape");
  if (n < 0 || n > (int64_t)INT_MAX / 8) return fail(NNM_E_INVAL, "n = %lld", (long long)n);
  if (!params || !dparams || (n > 0 && !x)) return fail(NNM_E_INVAL, "null argument");
  int dev;
  if (current_device(&dev) != NNM_OK) return NNM_E_DEVICE;
  const int grid = fit_fb_grid(shape->width, dev);
  const FitLayout FL = fit_layout(*shape, n, grid);
  if (!workspace || workspace_bytes < (int64_t)FL.total)
    return fail(NNM_E_INVAL, "workspace of %lld bytes, %zu needed", (long long)workspace_bytes, FL.total);
  return fit_backward_impl(*shape, params, dev, grid, (char*)workspace, FL, 1, n, 0, x, nullptr, nullptr, nullptr,
                           dvalue, dgrad, nullptr, dparams, dx, (hipStream_t)stream);
}

int fit_create(const nnm_net_shape* shape, const float* params, int device, int64_t max_points, nnm_fit** out) {
  g_err.clear();
  if (!out) return fail(NNM_E_INVAL, "null output handle");
  *out = nullptr;
  if (!shape_ok(shape)) return fail(NNM_E_UNSUPPORTED, "unsupported network shape");
  if (!params) return fail(NNM_E_INVAL, "null params");
  if (max_points < 1 || max_points > (int64_t)INT_MAX / 8) return fail(NNM_E_INVAL, "max_points %lld", (long long)max_points);
  const int64_t P = param_count(shape->d_in, shape->width, shape->n_sine);
  for (int64_t k = 0; k < P; ++k)
    if (!std::isfinite(params[k])) return fail(NNM_E_NONFINITE, "non-finite parameter %lld", (long long)k);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(NNM_E_INVAL, "device %d", device);
  DeviceGuard guard(device);
  nnm_fit* f = new nnm_fit();
  f->device = device;
  f->shape = *shape;
  f->n_params = P;
  f->max_points = max_points;
  f->grid = fit_fb_grid(shape->width, device);
  f->layout = fit_layout(*shape, max_points, f->grid);
  hipError_t e;
  if ((e = hipMalloc((void**)&f->state, (size_t)P * 4 * 4)) != hipSuccess ||
      (e = hipMalloc((void**)&f->ws, f->layout.total)) != hipSuccess) {
    fit_free(f);
    return fail(NNM_E_NOMEM, "fit allocation (%zu bytes): %s", f->layout.total, hipGetErrorString(e));
  }
  if ((e = hipMemcpy(f->state, params, (size_t)P * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemset(f->state + P, 0, (size_t)P * 4 * 3)) != hipSuccess) {
    fit_free(f);
    return hip_fail(e, "fit upload");
  }
  *out = f;
  return NNM_OK;
}

void fit_free(nnm_fit* f) {
  if (!f) return;
  DeviceGuard guard(f->device);
  if (f->state) (void)hipFree(f->state);
  if (f->ws) (void)hipFree(f->ws);
  delete f;
}

static int fit_check_batch(const nnm_fit* f, const nnm_fit_batch* b) {
  if (!f || !b) return fail(NNM_E_INVAL, "null argument");
  if (b->n_surf < 0 || b->n_unif < 0) return fail(NNM_E_INVAL, "negative batch size");
  const int64_t n = b->n_surf + b->n_unif;
  if (n > f->max_points) return fail(NNM_E_INVAL, "batch of %lld points exceeds max_points %lld", (long long)n,
                                     (long long)f->max_points);
  if (b->n_surf > 0 && (!b->surf_x || !b->surf_n)) return fail(NNM_E_INVAL, "null surface arrays");
  if (b->n_unif > 0 && (!b->unif_x || !b->unif_sdf)) return fail(NNM_E_INVAL, "null uniform arrays");
  if (f->shape.d_in != 3) return fail(NNM_E_UNSUPPORTED, "the fitting loss takes 3-D points");
  return NNM_OK;
}

int fit_loss_grad(nnm_fit* f, const nnm_fit_batch* b, float* loss4, float* dparams, void* stream) {
  g_err.clear();
  int rc = fit_check_batch(f, b);
  if (rc != NNM_OK) return rc;
  if (!dparams) return fail(NNM_E_INVAL, "null dparams");
  DeviceGuard guard(f->device);
  const int64_t n = b->n_surf + b->n_unif;
  const FitLayout FL = fit_layout(f->shape, n, f->grid);
  return fit_backward_impl(f->shape, f->state, f->device, f->grid, f->ws, FL, 0, n, b->n_surf, b->surf_x, b->unif_x,
                           b->surf_n, b->unif_sdf, nullptr, nullptr, loss4, dparams, nullptr,
                           (hipStream_t)stream);
}

int fit_step(nnm_fit* f, const nnm_fit_batch* b, const nnm_adam* opt, float* loss4, void* stream) {
  g_err.clear();
  if (!opt) return fail(NNM_E_INVAL, "null optimiser parameters");
  if (!(opt->lr > 0.f) || !(opt->beta1 >= 0.f && opt->beta1 < 1.f) || !(opt->beta2 >= 0.f && opt->beta2 < 1.f) ||
      !(opt->eps > 0.f))
    return fail(NNM_E_INVAL, "bad Adam parameters");
  int rc = fit_check_batch(f, b);
  if (rc != NNM_OK) return rc;
  DeviceGuard guard(f->device);
  const int64_t P = f->n_params;
  float* params = f->state;
  float* m = f->state + P;
  float* v = f->state + 2 * P;
  float* grad = f->state + 3 * P;
  const int64_t n = b->n_surf + b->n_unif;
  const FitLayout FL = fit_layout(f->shape, n, f->grid);
  hipStream_t st = (hipStream_t)stream;
  rc = fit_backward_impl(f->shape, params, f->device, f->grid, f->ws, FL, 0, n, b->n_surf, b->surf_x, b->unif_x,
                         b->surf_n, b->unif_sdf, nullptr, nullptr, loss4, grad, nullptr, st);
  if (rc != NNM_OK) return rc;
  const int64_t t = f->step + 1;
  const double bc1 = 1.0 - std::pow((double)opt->beta1, (double)t);
  const double bc2 = 1.0 - std::pow((double)opt->beta2, (double)t);
  const hipError_t e = launch_adam(params, grad, m, v, P, opt->lr, opt->beta1, opt->beta2, opt->eps, (float)bc1,
                                   (float)bc2, st);
  if (e != hipSuccess) return hip_fail(e, "adam");
  f->step = t;
  return NNM_OK;
}

int fit_state(nnm_fit* f, float** params, float** adam_m, float** adam_v, int64_t* n_params) {
  if (!f) return fail(NNM_E_INVAL, "null fit");
  if (params) *params = f->state;
  if (adam_m) *adam_m = f->state + f->n_params;
  if (adam_v) *adam_v = f->state + 2 * f->n_params;
  if (n_params) *n_params = f->n_params;
  return NNM_OK;
}

int fit_export(nnm_fit* f, const char* path) {
  g_err.clear();
  if (!f || !path) return fail(NNM_E_INVAL, "null fit or path");
  std::vector<float> host;
  try {
    host.resize((size_t)f->n_params);
  } catch (...) {
    return fail(NNM_E_NOMEM, "host buffer");
  }
  int rc = fit_read_state(f, host.data(), nullptr, nullptr);
  if (rc != NNM_OK) return rc;
  return nnm_write_net_file(path, f->shape.d_in, f->shape.width, f->shape.n_sine, host.data(), f->n_params);
}

int fit_read_state(nnm_fit* f, float* params, float* adam_m, float* adam_v) {
  if (!f) return fail(NNM_E_INVAL, "null fit");
  DeviceGuard guard(f->device);
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "synchronize");
  const size_t bytes = (size_t)f->n_params * 4;
  float* dst[3] = {params, adam_m, adam_v};
  for (int i = 0; i < 3; ++i)
    if (dst[i] && (e = hipMemcpy(dst[i], f->state + i * f->n_params, bytes, hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail(e, "read state");
  return NNM_OK;
}

int fit_write_state(nnm_fit* f, const float* params, const float* adam_m, const float* adam_v) {
  if (!f) return fail(NNM_E_INVAL, "null fit");
  DeviceGuard guard(f->device);
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "synchronize");
  const size_t bytes = (size_t)f->n_params * 4;
  const float* src[3] = {params, adam_m, adam_v};
  for (int i = 0; i < 3; ++i)
    if (src[i] && (e = hipMemcpy(f->state + i * f->n_params, src[i], bytes, hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "write state");
  return NNM_OK;
}

int64_t fit_get_step(const nnm_fit* f) { return f ? f->step : -1; }

int fit_set_step(nnm_fit* f, int64_t step) {
  if (!f || step < 0) return fail(NNM_E_INVAL, "bad argument");
  f->step = step;
  return NNM_OK;
}

}  // extern "C"

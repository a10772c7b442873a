// fit_kernels.hip -- fitting a SIREN through its analytic gradient (double
// backward) on gfx950, in float32.
//
// Two launches per batch of points over the same tiles (8 points x the four
// columns [h | G_x G_y G_z] per wave, the tangent mode of the evaluator):
//   forward   layer by layer with the shared-forward tangent (Alg. 2 in the
//             G_i form), writing each layer's pre-activations (revolutions)
//             and inputs to a workspace laid out [column][neuron];
//   adjoints  of the loss terms, or the caller's upstream adjoints (end of
//             the forward launch, one value per column);
//   reverse   (second launch) through primal and tangent:
//               abar_i  = cos(a_i) hbar_{i+1} - sin(a_i) sum_j Tbar_{i+1,j} dA_{i,j}
//               dAbar_i = cos(a_i) Tbar_{i+1}
//               [hbar_i | Tbar_i] = W_i^T [abar_i | dAbar_i]   (32x32x2 MFMAs)
//             overwriting the pre-activations with [abar_i | dAbar_i].
// The parameter gradient is then W_i-bar = sum over columns [abar|dAbar] X^T:
// reductions over the workspace (split-K MFMA GEMM and column reductions).
#include "nnm_kernels.h"
#include "siren_tile.h"

namespace nnm {

constexpr float kTwoPiF = 6.28318530717958647692f;

// Sum over the four lanes of each quad.
__device__ inline float quad_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));  // [1,0,3,2]
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));  // [2,3,0,1]
  return v;
}

// ------------------------------------------------------------ packing (fp32)
// Flat parameters (row major [out][in] per layer) -> the layouts the tile uses.
__global__ void k_fit_pack(FitPackArgs A) {
  const int H = A.width, K = A.n_sine, MB = H / 32, d_in = A.d_in;
  const long long n_a0 = 3LL * MB * 64;
  const long long n_bh = (long long)(K - 1) * H;
  const long long n_wk = H;
  const long long n_ah = (long long)(K - 1) * H * H;  // per copy (forward, transposed)
  const long long total = n_a0 + n_bh + n_wk + 2 * n_ah + H + 1;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    long long i = e;
    if (i < n_a0) {
      const int lane = (int)(i % 64), mb = (int)((i / 64) % MB), ks = (int)(i / (64 * MB));
      const int row = 32 * mb + lane % 32, k = 2 * ks + lane / 32;
      float v = 0.f;
      if (k < d_in)
        v = A.params[A.w_off[0] + (long long)row * d_in + k];
      else if (k == d_in)
        v = A.params[A.b_off[0] + row];
      A.a0[i] = v / kTwoPiF;
      continue;
    }
    i -= n_a0;
    if (i < n_bh) {
      const int layer = 1 + (int)(i / H), slot = (int)(i % H);
      const int mb = slot / 32, g = (slot / 16) % 2, r = slot % 16;
      A.bh[i] = A.params[A.b_off[layer] + acc_row(mb, g, r)] / kTwoPiF;
      continue;
    }
    i -= n_bh;
    if (i < n_wk) {
      const int slot = (int)i, mb = slot / 32, g = (slot / 16) % 2, r = slot % 16;
      A.wk[i] = A.params[A.w_off[K] + acc_row(mb, g, r)];
      continue;
    }
    i -= n_wk;
    if (i < 2 * n_ah) {
      const bool transposed = i >= n_ah;
      const long long j = transposed ? i - n_ah : i;
      const int layer = 1 + (int)(j / ((long long)H * H));
      const long long w = j % ((long long)H * H);
      // f32x4 group (q, mb, lane), element e
      const int e4 = (int)(w % 4), lane = (int)((w / 4) % 64), mb = (int)((w / 256) % MB), q = (int)(w / (256 * MB));
      const int ks = 4 * q + e4, row = 32 * mb + lane % 32, kn = kperm_2(ks, lane / 32);
      const long long base = A.w_off[layer];
      if (!transposed)
        A.ah[j] = A.params[base + (long long)row * H + kn] / kTwoPiF;
      else
        A.aht[j] = A.params[base + (long long)kn * H + row];  // W^T[row = input][k = output]
      continue;
    }
    i -= 2 * n_ah;
    if (i < H) {
      const int slot = (int)i, mb = slot / 32, g = (slot / 16) % 2, r = slot % 16, row = acc_row(mb, g, r);
      const long long b = A.w_off[0] + (long long)row * d_in;
      A.w0t[i] = make_float4(A.params[b], A.params[b + 1], A.params[b + 2], d_in == 4 ? A.params[b + 3] : 0.f);
      continue;
    }
    A.bk[0] = A.params[A.b_off[K]];
  }
}

#ifndef NNM_FIT_BWD_PRE
#define NNM_FIT_BWD_PRE 4
#endif
// ------------------------------------------------ forward, then reverse
// Two launches over the same tile-to-wave map: FWD runs the forward pass and
// the loss adjoints (written to adj), the reverse launch starts from adj.  As
// one kernel the two phases' register states overlap and spill.
template <int H, bool FWD>
__global__ void __launch_bounds__(kBlockThreads) k_fit_fb(FitArgs A) {
  constexpr int MB = H / 32;
  __shared__ NetSmem<H> sm;
  __shared__ float4 s_w0t[FWD ? 1 : H];
  stage_net<H>(&sm, A.L);
  if (!FWD)
    for (int i = threadIdx.x; i < H; i += blockDim.x) s_w0t[i] = A.w0t[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int col = lane & 31;
  const int g = lane >> 5;
  const int q = col >> 2, c = col & 3;
  const int waves = kBlockThreads / 64;
  const int wave = blockIdx.x * waves + (threadIdx.x >> 6);
  const int nwaves = gridDim.x * waves;
  const int ntiles = (A.n + 7) / 8;
  const long long Kc = A.Kc;
  const int K = A.L.n_sine;
  SirenTile<H, PREC_FP32, true> tile;
  float lsum[4] = {0.f, 0.f, 0.f, 0.f};
  for (int t = wave; t < ntiles; t += nwaves) {
    const int p = t * 8 + q;
    const bool live = p < A.n;
    const long long gcol = (long long)t * 32 + col;
    if constexpr (FWD) {
    // ---- inputs
    const float* xp = nullptr;
    bool surf = false;
    if (live) {
      if (A.mode == 0) {
        surf = p < A.n_surf;
        xp = surf ? A.x0 + 3LL * p : A.x1 + 3LL * (p - A.n_surf);
      } else {
        xp = A.x0 + (long long)A.L.d_in * p;
      }
    }
    float4 in = make_float4(0.f, 0.f, 0.f, 0.f);
    if (xp) {
      in.x = xp[0];
      in.y = xp[1];
      in.z = xp[2];
      if (A.L.d_in == 4) in.w = xp[3];
    }
    // ---- forward: store pre-activations (revolutions) and layer inputs
    NNM_MEM_FENCE();
    for (int layer = 0; layer < K; ++layer) {
      // acc is born inside the iteration: live across the back edge are only
      // the activations, which keeps the forward within the register file.
      f32x16_t acc[MB];
      if (layer == 0)
        tile.layer0_acc(&sm, A.L, in, c, acc);
      else
        tile.hidden_acc(&sm, A.L, layer, c, acc);
      // [column][neuron] slabs: rows 32 mb + 8 b + 4 g .. +3 are 16 contiguous bytes
      float4* pa = (float4*)(A.ws_abar + ((long long)layer * Kc + gcol) * H + 4 * g);
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          pa[(32 * mb + 8 * b) / 4] = make_float4(acc[mb][4 * b], acc[mb][4 * b + 1], acc[mb][4 * b + 2], acc[mb][4 * b + 3]);
      tile.activate(acc, c, layer == 0 || A.L.reduce_hidden != 0);
      float4* px = (float4*)(A.ws_x + ((long long)layer * Kc + gcol) * H + 4 * g);
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          px[(32 * mb + 8 * b) / 4] = make_float4(tile.act[mb][4 * b], tile.act[mb][4 * b + 1], tile.act[mb][4 * b + 2],
                                                  tile.act[mb][4 * b + 3]);
    }
    const float val = tile.output(&sm, A.L, c);
    const float N = quad_bcast<0>(val), gx = quad_bcast<1>(val), gy = quad_bcast<2>(val),
                gz = quad_bcast<3>(val);
    // ---- adjoints dL/dN, dL/dgrad N of this point
    float Nbar = 0.f, gb[3] = {0.f, 0.f, 0.f};
    if (live) {
      if (A.mode == 0) {
        if (surf) {
          const float* np_ = A.surf_n + 3LL * p;
          const float nx = np_[0], ny = np_[1], nz = np_[2];
          Nbar = (N > 0.f ? 1.f : (N < 0.f ? -1.f : 0.f)) * A.inv_ns;
          // normal term on the unit gradient, 1 - n . u with u = grad N / |grad N|:
          // adjoint -(n - (n . u) u) / |grad N| (zero for a zero gradient)
          const float gn = sqrtf(gx * gx + gy * gy + gz * gz);
          const float ig = gn > 0.f ? 1.f / gn : 0.f;
          const float cs = (nx * gx + ny * gy + nz * gz) * ig;
          gb[0] = -(nx - cs * gx * ig) * ig * A.inv_ns;
          gb[1] = -(ny - cs * gy * ig) * ig * A.inv_ns;
          gb[2] = -(nz - cs * gz * ig) * ig * A.inv_ns;
          if (c == 0 && g == 0) {
            lsum[0] += fabsf(N);
            lsum[1] += 1.f - cs;
          }
        } else {
          const float sdf = A.unif_sdf[p - A.n_surf];
          const float dlt = N - sdf;
          Nbar = (dlt > 0.f ? 1.f : (dlt < 0.f ? -1.f : 0.f)) * A.inv_nu;
          const float gn = sqrtf(gx * gx + gy * gy + gz * gz);
          const float s = gn > 0.f ? 2.f * (gn - 1.f) / gn * A.inv_nu : 0.f;
          gb[0] = s * gx;
          gb[1] = s * gy;
          gb[2] = s * gz;
          if (c == 0 && g == 0) {
            lsum[2] += fabsf(dlt);
            lsum[3] += (gn - 1.f) * (gn - 1.f);
          }
        }
      } else {
        Nbar = A.dvalue ? A.dvalue[p] : 0.f;
        if (A.dgrad) {
          gb[0] = A.dgrad[3LL * p];
          gb[1] = A.dgrad[3LL * p + 1];
          gb[2] = A.dgrad[3LL * p + 2];
        }
      }
    }
    const float adjc = (c == 0) ? Nbar : (c == 1 ? gb[0] : (c == 2 ? gb[1] : gb[2]));
    if (g == 0) A.adj[gcol] = adjc;
    } else {
    // ---- reverse: X-bar of the output layer, then layer by layer
    const float adjc = A.adj[gcol];
    NNM_MEM_FENCE();
    float xbar[MB][16];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int r = 0; r < 16; ++r) xbar[mb][r] = sm.wk[acc_slot(mb, g, r)] * adjc;
    for (int layer = K - 1; layer >= 0; --layer) {
      float4* pa = (float4*)(A.ws_abar + ((long long)layer * Kc + gcol) * H + 4 * g);
      const bool reduce = layer == 0 || A.L.reduce_hidden;
      NNM_MEM_FENCE();
      // Slab loads run kPre row blocks ahead of their use at H = 256 (a single
      // wave per SIMD hides no latency by itself; narrower widths run two or
      // more waves per SIMD and load at the point of use).
      constexpr int kPre = H >= 256 ? NNM_FIT_BWD_PRE : 0;
      float4 pv[MB][4];  // primal: a / 2pi; tangent: dA / 2pi
#pragma unroll
      for (int mb = 0; mb < kPre; ++mb)
#pragma unroll
        for (int b = 0; b < 4; ++b) pv[mb][b] = pa[(32 * mb + 8 * b) / 4];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb) {
        if (mb + kPre < MB) {
#pragma unroll
          for (int b = 0; b < 4; ++b) pv[mb + kPre][b] = pa[(32 * (mb + kPre) + 8 * b) / 4];
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const float4 v4 = pv[mb][b];
          const float vv[4] = {v4.x, v4.y, v4.z, v4.w};
          float ab4[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int r = 4 * b + i;
            const float v = vv[i];
            float rp = quad_bcast<0>(v);
            if (reduce) rp = fract_rev(rp);
            const float cs = cos_rev(rp), sn = sin_rev(rp);
            const float xb = xbar[mb][r];
            const float prod = (c == 0) ? 0.f : xb * (kTwoPiF * v);  // Tbar_j dA_j
            const float ssum = quad_sum(prod);
            const float ab = (c == 0) ? fmaf(cs, xb, -sn * ssum) : cs * xb;
            ab4[i] = ab;
            xbar[mb][r] = ab;  // now [abar | dAbar] of this layer
          }
          pa[(32 * mb + 8 * b) / 4] = make_float4(ab4[0], ab4[1], ab4[2], ab4[3]);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      if (layer > 0) {
        f32x16_t nb[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int r = 0; r < 16; ++r) nb[mb][r] = 0.f;
        const f32x4_t* AT = (const f32x4_t*)((const char*)A.aht + (long long)(layer - 1) * H * H * 4);
        gemm_fp32<H>(xbar, AT, nb);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int r = 0; r < 16; ++r) xbar[mb][r] = nb[mb][r];
      } else if (A.dx) {
        // dL/dx through N: W_0^T abar_0 (primal column; the tangent seeds are constant)
        float d4[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const float4 w = s_w0t[acc_slot(mb, g, r)];
            const float ab = xbar[mb][r];
            d4[0] = fmaf(w.x, ab, d4[0]);
            d4[1] = fmaf(w.y, ab, d4[1]);
            d4[2] = fmaf(w.z, ab, d4[2]);
            d4[3] = fmaf(w.w, ab, d4[3]);
          }
#pragma unroll
        for (int j = 0; j < 4; ++j) d4[j] += __shfl_xor(d4[j], 32);
        if (c == 0 && g == 0 && live)
          for (int j = 0; j < A.L.d_in; ++j) A.dx[(long long)A.L.d_in * p + j] = d4[j];
      }
    }
    }
  }
  // per-wave loss partial sums (deterministic: fixed tile to wave map)
  if (FWD && A.loss_part) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      float v = lsum[j];
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      if (lane == 0) A.loss_part[4LL * wave + j] = v;
    }
  }
}

// Column weights for the layer-0 gradient: w_j[col] = x_j (primal column), 1 on
// the tangent column of coordinate j, else 0; plus the primal mask.
__global__ void k_fit_vectors(FitVecArgs A) {
  const long long Kc = A.Kc;
  for (long long col = blockIdx.x * (long long)blockDim.x + threadIdx.x; col < Kc;
       col += (long long)gridDim.x * blockDim.x) {
    const long long p = col / 4;
    const int c = (int)(col % 4);
    float x[4] = {0.f, 0.f, 0.f, 0.f};
    if (p < A.n) {
      const float* xp;
      if (A.mode == 0)
        xp = p < A.n_surf ? A.x0 + 3 * p : A.x1 + 3 * (p - A.n_surf);
      else
        xp = A.x0 + (long long)A.d_in * p;
      for (int j = 0; j < A.d_in; ++j) x[j] = xp[j];
    }
    const bool live = p < A.n;
    A.mask[col] = (c == 0 && live) ? 1.f : 0.f;
    for (int j = 0; j < A.d_in; ++j) {
      float w = 0.f;
      if (live) {
        if (c == 0)
          w = x[j];
        else if (j < 3 && c == j + 1)
          w = 1.f;
      }
      A.wvec[(long long)j * Kc + col] = w;
    }
  }
}

// Sums the per-wave loss partials in a fixed order (one block).
__global__ void k_fit_loss_reduce(const float* part, int nwaves, float inv_ns, float inv_nu, float* loss4) {
  __shared__ float sh[4][256];
  const int t = threadIdx.x;
  float s[4] = {0.f, 0.f, 0.f, 0.f};
  for (int w = t; w < nwaves; w += blockDim.x)
    for (int j = 0; j < 4; ++j) s[j] += part[4LL * w + j];
  for (int j = 0; j < 4; ++j) sh[j][t] = s[j];
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (t < off)
      for (int j = 0; j < 4; ++j) sh[j][t] += sh[j][t + off];
    __syncthreads();
  }
  if (t == 0) {
    loss4[0] = sh[0][0] * inv_ns;
    loss4[1] = sh[1][0] * inv_ns;
    loss4[2] = sh[2][0] * inv_nu;
    loss4[3] = sh[3][0] * inv_nu;
  }
}

// Adam (Kingma & Ba): m, v moments; bias corrections bc1 = 1 - beta1^t,
// bc2 = 1 - beta2^t computed by the host in float64.
__global__ void k_adam(float* params, const float* grad, float* m, float* v, long long n, float lr, float b1,
                       float b2, float eps, float bc1, float bc2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const float gi = grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / bc1, vh = vi / bc2;
    params[i] -= lr * mh / (sqrtf(vh) + eps);
  }
}

// ------------------------------------------- weight-gradient reductions
// Column reduction over a [Kc][H] slab, restricted to the columns
// col = j * cstep (a weight vector that vanishes elsewhere by construction,
// such as the primal mask, lets the other columns go unread).  First pass:
// block b takes the stepped columns j in [b * per_blk, (b + 1) * per_blk) and
// writes part[b][r][row] = sum_j M[j cstep][row] w_r[j cstep].  A thread owns
// four consecutive rows of one column (one 16-byte load); the block covers
// 1024 / H columns per pass and keeps kColU passes of loads in flight.  The
// per-thread sums are combined in LDS in a fixed order, so results do not
// depend on scheduling.
constexpr int kColU = 8;
template <int R>
__global__ void __launch_bounds__(256) k_colreduce(const float* __restrict__ M, int H, long long Kc,
                                                   const float* __restrict__ w, int cstep, long long per_blk,
                                                   float* __restrict__ part) {
  __shared__ float4 sh[R][256];  // [r][sub * H / 4 + q]
  const int tid = threadIdx.x;
  const int lq = H >> 2;         // threads per column
  const int cpi = 256 / lq;      // columns per block pass
  const int sub = tid / lq, q = tid - sub * lq;
  const long long nsc = (Kc + cstep - 1) / cstep;
  const long long j0 = (long long)blockIdx.x * per_blk;
  const long long j1 = min(j0 + per_blk, nsc);
  float4 acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = make_float4(0.f, 0.f, 0.f, 0.f);
  const float4* M4 = reinterpret_cast<const float4*>(M);
  long long j = j0 + sub;
  for (; j + (long long)(kColU - 1) * cpi < j1; j += (long long)kColU * cpi) {
    float4 m[kColU];
    float wv[kColU][R];
#pragma unroll
    for (int u = 0; u < kColU; ++u) {
      const long long col = (j + (long long)u * cpi) * cstep;
      m[u] = M4[col * lq + q];
#pragma unroll
      for (int r = 0; r < R; ++r) wv[u][r] = w[r * Kc + col];
    }
#pragma unroll
    for (int u = 0; u < kColU; ++u)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        acc[r].x = fmaf(m[u].x, wv[u][r], acc[r].x);
        acc[r].y = fmaf(m[u].y, wv[u][r], acc[r].y);
        acc[r].z = fmaf(m[u].z, wv[u][r], acc[r].z);
        acc[r].w = fmaf(m[u].w, wv[u][r], acc[r].w);
      }
  }
  for (; j < j1; j += cpi) {
    const long long col = j * cstep;
    const float4 m = M4[col * lq + q];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float wr = w[r * Kc + col];
      acc[r].x = fmaf(m.x, wr, acc[r].x);
      acc[r].y = fmaf(m.y, wr, acc[r].y);
      acc[r].z = fmaf(m.z, wr, acc[r].z);
      acc[r].w = fmaf(m.w, wr, acc[r].w);
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) sh[r][tid] = acc[r];
  __syncthreads();
  const float* shf = reinterpret_cast<const float*>(&sh[0][0]);
  for (int o = tid; o < R * H; o += 256) {
    const int r = o / H, row = o - r * H;
    float s = 0.f;
    for (int c = 0; c < cpi; ++c) s += shf[r * 1024 + c * H + row];
    part[((long long)blockIdx.x * R + r) * H + row] = s;
  }
}

// Second pass: dst_r[row * stride_r] = sum over the nblk first-pass blocks of
// part[b][r][row].  Block (64 rows) x (16 interleaved groups of blocks); the
// groups are added in a fixed order.
__global__ void __launch_bounds__(1024) k_colreduce_final(const float* __restrict__ part, int nblk, int R, int H,
                                                          ColDst dst) {
  __shared__ float sh[16][64];
  const int x = threadIdx.x & 63, y = threadIdx.x >> 6;
  const int row = blockIdx.x * 64 + x;
  const int r = blockIdx.y;
  float s = 0.f;
  if (row < H) {
#pragma unroll 8
    for (int c = y; c < nblk; c += 16) s += part[((long long)c * R + r) * H + row];
  }
  sh[y][x] = s;
  __syncthreads();
  if (y == 0 && row < H) {
    float t = 0.f;
#pragma unroll
    for (int g = 0; g < 16; ++g) t += sh[g][x];
    dst.ptr[r][(long long)row * dst.stride[r]] = t;
  }
}

// Weight gradient of a hidden layer, split over column chunks:
// part[chunk][o][i] = sum_{col in chunk} abar[col][o] X[col][i] (32x32x2 fp32
// MFMAs).  One wave per 32-row block of the output, each accumulating against
// every 32-column block (H/32 accumulator tiles: two waves fit a SIMD at
// H = 256, so one loads while the other multiplies).  Each iteration issues
// all loads of kWgradU column pairs before the first of their MFMAs (left to
// itself the scheduler spreads the loads between the MFMAs, and the late ones
// expose their latency).
constexpr int kWgradU = 4;
template <int H>
__global__ void __launch_bounds__(2 * H) k_wgrad(const float* __restrict__ abar, const float* __restrict__ X,
                                                 long long Kc, int chunk, float* __restrict__ part) {
  constexpr int MB = H / 32;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane & 31, g = lane >> 5;
  f32x16_t acc[MB];
#pragma unroll
  for (int b = 0; b < MB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[b][r] = 0.f;
  const long long c0 = (long long)blockIdx.x * chunk;
  const long long c1 = min(c0 + chunk, Kc);
  // Kc and chunk are multiples of 2 kWgradU, so every batch is whole.
  for (long long col = c0; col < c1; col += 2 * kWgradU) {
    float av[kWgradU], bv[kWgradU][MB];
#pragma unroll
    for (int u = 0; u < kWgradU; ++u) {
      const long long cg = col + 2 * u + g;
      av[u] = abar[cg * H + 32 * wave + i];
#pragma unroll
      for (int b = 0; b < MB; ++b) bv[u][b] = X[cg * H + 32 * b + i];
    }
    __builtin_amdgcn_sched_barrier(0);  // every load of the batch issues before the first MFMA
#pragma unroll
    for (int u = 0; u < kWgradU; ++u)
#pragma unroll
      for (int b = 0; b < MB; ++b) acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[u], bv[u][b], acc[b], 0, 0, 0);
  }
  float* out = part + (long long)blockIdx.x * H * H;
#pragma unroll
  for (int b = 0; b < MB; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int o = 32 * wave + 8 * (r / 4) + 4 * g + (r % 4);
      out[(long long)o * H + 32 * b + i] = acc[b][r];
    }
}

__global__ void k_wgrad_final(const float* __restrict__ part, int nchunk, long long HH, float* __restrict__ dst) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < HH; e += (long long)gridDim.x * blockDim.x) {
    float s = 0.f;
#pragma unroll 8
    for (int c = 0; c < nchunk; ++c) s += part[(long long)c * HH + e];
    dst[e] = s;
  }
}

// Sum of a[j cstep] m[j cstep] over the stepped columns: block b sums the range
// [b per_blk, (b + 1) per_blk) into part[b] (fixed-order tree), then one block
// adds the partial sums in a fixed order.
__global__ void __launch_bounds__(256) k_masked_sum(const float* __restrict__ a, const float* __restrict__ m,
                                                    long long n, int cstep, long long per_blk,
                                                    float* __restrict__ part) {
  __shared__ float sh[256];
  const long long nsc = (n + cstep - 1) / cstep;
  const long long j0 = (long long)blockIdx.x * per_blk, j1 = min(j0 + per_blk, nsc);
  float s = 0.f;
  for (long long j = j0 + threadIdx.x; j < j1; j += 256) s = fmaf(a[j * cstep], m[j * cstep], s);
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(256) k_sum_final(const float* __restrict__ part, int nblk, float* out) {
  __shared__ float sh[256];
  float s = 0.f;
  for (int b = threadIdx.x; b < nblk; b += 256) s += part[b];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// ------------------------------------------------------------------ launchers

int colreduce_blocks(long long ncols, int H) {
  const long long cpi = 1024 / H;
  return (int)std::max<long long>(1, std::min<long long>(kColBlocks, (ncols + cpi - 1) / cpi));
}

hipError_t launch_colreduce(const float* M, int H, long long Kc, const float* w, int R, int cstep, float* part,
                            const ColDst& dst, hipStream_t s) {
  if (H < 32 || H > 256 || (H & 31) || cstep < 1 || Kc < 1) return hipErrorInvalidValue;
  const long long nsc = (Kc + cstep - 1) / cstep;
  int nblk = colreduce_blocks(nsc, H);
  const long long per_blk = (nsc + nblk - 1) / nblk;
  nblk = (int)((nsc + per_blk - 1) / per_blk);
  switch (R) {
#define NNM_COLRED(RR)                                                                                       \
  case RR:                                                                                                  \
    hipLaunchKernelGGL(k_colreduce<RR>, dim3(nblk), dim3(256), 0, s, M, H, Kc, w, cstep, per_blk, part); \
    break;
    NNM_COLRED(1)
    NNM_COLRED(2)
    NNM_COLRED(4)
    NNM_COLRED(5)
#undef NNM_COLRED
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_colreduce_final, dim3((H + 63) / 64, R), dim3(1024), 0, s, part, nblk, R, H, dst);
  return hipGetLastError();
}

hipError_t launch_wgrad(int H, const float* abar, const float* X, long long Kc, int chunk, float* part, float* dst,
                        hipStream_t s) {
  constexpr int kStep = 2 * kWgradU;
  if (Kc % kStep || chunk % kStep || chunk < kStep || Kc < kStep) return hipErrorInvalidValue;
  const int nchunk = (int)((Kc + chunk - 1) / chunk);
  switch (H) {
    case 32: hipLaunchKernelGGL(k_wgrad<32>, dim3(nchunk), dim3(64), 0, s, abar, X, Kc, chunk, part); break;
    case 64: hipLaunchKernelGGL(k_wgrad<64>, dim3(nchunk), dim3(128), 0, s, abar, X, Kc, chunk, part); break;
    case 128: hipLaunchKernelGGL(k_wgrad<128>, dim3(nchunk), dim3(256), 0, s, abar, X, Kc, chunk, part); break;
    case 256: hipLaunchKernelGGL(k_wgrad<256>, dim3(nchunk), dim3(512), 0, s, abar, X, Kc, chunk, part); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long HH = (long long)H * H;
  hipLaunchKernelGGL(k_wgrad_final, dim3((int)std::min<long long>((HH + 255) / 256, 1024)), dim3(256), 0, s, part,
                     nchunk, HH, dst);
  return hipGetLastError();
}

hipError_t launch_masked_sum(const float* a, const float* m, long long n, int cstep, float* part, float* out,
                             hipStream_t s) {
  if (cstep < 1 || n < 1) return hipErrorInvalidValue;
  const long long nsc = (n + cstep - 1) / cstep;
  int nblk = (int)std::min<long long>(kSumBlocks, (nsc + 255) / 256);
  const long long per_blk = (nsc + nblk - 1) / nblk;
  nblk = (int)((nsc + per_blk - 1) / per_blk);
  hipLaunchKernelGGL(k_masked_sum, dim3(nblk), dim3(256), 0, s, a, m, n, cstep, per_blk, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, part, nblk, out);
  return hipGetLastError();
}


hipError_t launch_fit_pack(const FitPackArgs& a, hipStream_t s) {
  const long long H = a.width, K = a.n_sine;
  const long long total = 3 * (H / 32) * 64 + (K - 1) * H + H + 2 * (K - 1) * H * H + H + 1;
  const int grid = (int)std::min<long long>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fit_pack, dim3(grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fit_fb(const FitArgs& a, int grid, hipStream_t s) {
#define NNM_FIT_FB(HH)                                                                    \
  case HH:                                                                                \
    hipLaunchKernelGGL((k_fit_fb<HH, true>), dim3(grid), dim3(kBlockThreads), 0, s, a);  \
    if (hipGetLastError() != hipSuccess) break;                                           \
    hipLaunchKernelGGL((k_fit_fb<HH, false>), dim3(grid), dim3(kBlockThreads), 0, s, a); \
    break;
  switch (a.L.width) {
    NNM_FIT_FB(32)
    NNM_FIT_FB(64)
    NNM_FIT_FB(128)
    NNM_FIT_FB(256)
    default: return hipErrorInvalidValue;
  }
#undef NNM_FIT_FB
  return hipGetLastError();
}

hipError_t launch_fit_vectors(const FitVecArgs& a, hipStream_t s) {
  const int grid = (int)std::min<long long>((a.Kc + 255) / 256, 8192);
  hipLaunchKernelGGL(k_fit_vectors, dim3(std::max(grid, 1)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fit_loss_reduce(const float* part, int nwaves, float inv_ns, float inv_nu, float* loss4,
                                  hipStream_t s) {
  hipLaunchKernelGGL(k_fit_loss_reduce, dim3(1), dim3(256), 0, s, part, nwaves, inv_ns, inv_nu, loss4);
  return hipGetLastError();
}

hipError_t launch_adam(float* params, const float* grad, float* m, float* v, long long n, float lr, float b1,
                       float b2, float eps, float bc1, float bc2, hipStream_t s) {
  const int grid = (int)std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_adam, dim3(std::max(grid, 1)), dim3(256), 0, s, params, grad, m, v, n, lr, b1, b2, eps, bc1,
                     bc2);
  return hipGetLastError();
}

int fit_fb_grid(int width, int device) {
  // both phases use the grid of the forward launch (the loss partial sums
  // are laid out per wave of that grid)
  const void* fn = width == 32 ? (const void*)k_fit_fb<32, true>
                   : width == 64 ? (const void*)k_fit_fb<64, true>
                   : width == 128 ? (const void*)k_fit_fb<128, true>
                                  : (const void*)k_fit_fb<256, true>;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlockThreads, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
  return per_cu * cus;
}

}  // namespace nnm

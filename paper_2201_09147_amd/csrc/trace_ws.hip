// trace_ws.hip -- pipelined weight-stationary tracing and normal kernels for
// width-256 networks with two hidden layers in bf16 / fp16 (the fine level of
// the nested stacks).
//
// A workgroup is eight waves in two teams, one workgroup per CU, and every SIMD
// holds one wave of each team (roles are assigned from the SIMD each wave runs
// on).  Team 1 (waves 0-3) keeps rows [64 w, 64 w + 64) of the first hidden
// weight matrix in registers for the whole kernel, team 2 (waves 4-7) the same
// rows of the second; the hidden weights are read from memory once per
// workgroup.  Tiles of 32 columns (32 rays) when tracing, 64 columns (16 points
// x [h | G_x G_y G_z], two 32-column MFMA blocks) in the normal pass, move
// through a software pipeline with one workgroup barrier per stage.  In stage s:
//   * every wave evaluates its 32-row block of the first sine layer of tile s
//     (32x32x2 fp32 MFMA over (x, y, z[, t], 1), then sin) into act0[s % 2];
//   * team 1 multiplies tile s-1 (act0) by its rows of W_1 (32x32x16 MFMAs,
//     B operand from LDS, C initialised with the bias), applies sin and writes
//     the 16-bit activations to act1[(s-1) % 2]: MFMA first, then VALU;
//   * team 2 applies sin to its accumulators of tile s-3 and forms its part of
//     the output dot product, then multiplies tile s-2 (act1) by its rows of
//     W_2: VALU first, then MFMA;
//   * role 0 (a team-1 wave, after its sines; role 1 takes over its
//     first-layer block) takes the outputs of tile s-4, runs the
//     Algorithm 1 update (or the normal's last step), retires finished rays,
//     refills the freed slots and writes the inputs of tile s+1.
// The two teams' MFMA and VALU phases are opposite, so each SIMD overlaps one
// wave's matrix work with the other's sines.  Tile t occupies slot group
// t % kPipeGroups; the ray state of a group waits in LDS while its tile is in
// flight.  Activations are exchanged in natural row order, so these kernels use
// the row-split fragments of the weight-stationary pack, not the K permutation
// of the single-wave tiles.
#include "trace_common.h"

namespace nnm {

constexpr int kPipeThreads = 512;
// Columns per tile: 32 for tracing (fewer rays in flight keeps the tiles full
// while the last, longest rays finish), 64 for the normal pass (no iteration,
// so twice the columns per control step is a straight gain).
constexpr int kTraceCols = NNM_WS_TRACE_COLS;
constexpr int kNormalCols = 64;
constexpr int kPipeStride = 256 + 8;  // 16-bit elements per LDS column (spreads LDS banks)
constexpr int kParkMax = kTraceCols / 2;  // most survivors a group parks (tail compaction)
// Tracing kernel: the control wave (role 0) computes no part of the first
// hidden product.  Its two W_1 row blocks live in LDS and roles 1 and 2 each
// compute one of them after their own, so the control wave's stage is the
// control alone; role 3 takes over the control wave's first-layer block.
#ifndef NNM_WS_CTL_NOH1
#define NNM_WS_CTL_NOH1 1
#endif
// tracing: the wave that computes role 0's first-layer block
constexpr int kOff0Wave = (kTraceCols == 32 && NNM_WS_CTL_NOH1) ? 3 : 1;
static_assert(kPipeGroups == 5, "tile t uses group t % 5: five tiles are in flight");
static_assert(kOrderKeys == 64, "the control wave keeps one order key per lane");
static_assert(kPipeGroups * kTraceCols == kWsRaysPerBlock && kPipeGroups * kNormalCols / 4 == kWsPointsPerBlock, "slots");

template <int C>
struct PipeSmem {
  // tracing kernel with NNM_WS_CTL_NOH1: the control wave's two W_1 row blocks
  // (2 blocks x 16 k-steps x 64 lanes of 16-byte fragments, 32 KB)
  uint4 w1lds[(C == 32 && NNM_WS_CTL_NOH1) ? 2 * 16 * 64 : 1];
  uint16_t act0[2][C * kPipeStride];
  uint16_t act1[2][C * kPipeStride];
  float bias[2][256];
  float zeros[256];
  float wk[256];
  float part[2][4][C];
  float4 xin[2][C];
  // slot records, three float4 per slot: tracing {o, tau} {v, t} {ray, k | st << 16, c(t)};
  // normal {x, 0} {c(t), 0, 0} {ray, 0, 0, 0}
  float4 srec[kPipeGroups][3][C];
  float4 park[3][C];  // tracing: parked slot records (tail compaction)
  int tlive[8];
  int stop[2];
  int simd_count[4];
  int role_of[8];
  int ring[2 * kPushBatch];          // tracing: finished rays waiting for the output queue
  uint8_t ring_key[2 * kPushBatch];  // tracing: their order keys
  int hist[kOrderKeys];              // tracing: pushed rays per order key
};

template <int P>
struct PipeBits;
template <>
struct PipeBits<PREC_BF16> {
  static __device__ inline uint16_t bits(float v) { return __builtin_bit_cast(uint16_t, (__bf16)v); }
};
template <>
struct PipeBits<PREC_FP16> {
  static __device__ inline uint16_t bits(float v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
};

// Per-lane roles.  TAN: column j = 4 q + c is point q's primal (c = 0) or
// tangent c column; the activation is sin(2 pi r) on primal columns and
// (2 pi v) cos(2 pi r) = (2 pi v) sin(2 pi (r + 1/4)) on tangent columns, r the
// quad's primal pre-activation: one sine and one fma per element.
struct PipeLane {
  int j, g, c;
  float off, m1, m0;
};

template <bool TAN>
__device__ inline PipeLane pipe_lane(int lane) {
  PipeLane p;
  p.j = lane & 31;
  p.g = lane >> 5;
  p.c = TAN ? (p.j & 3) : 0;
  p.off = p.c ? 0.25f : 0.f;
  p.m1 = p.c ? kTwoPi : 0.f;
  p.m0 = p.c ? 0.f : 1.f;
  return p;
}

template <bool TAN, bool RED>
__device__ inline float pipe_act(float v, const PipeLane& pl) {
  if (TAN) {
    float r = quad_bcast<0>(v) + pl.off;
    if (RED) r = fract_rev(r);
    return sin_rev(r) * fmaf(v, pl.m1, pl.m0);
  }
  return sin_rev(RED ? fract_rev(v) : v);
}

// Stationary registers of one wave: its 32-row block of the layer-0 operand
// and its 64 rows of its team's hidden matrix.
template <int P>
struct PipeWeights {
  typedef typename HiddenOps<P>::frag_t frag_t;
  float w0[2][3];  // the operands of the (up to two) first-layer row blocks this wave computes
  frag_t w[2][16];

  __device__ inline void load(const DevLevel& L, int wave, int lane, int blk0, int blk1) {
    const int team = wave >> 2, tw = wave & 3;
#pragma unroll
    for (int ks = 0; ks < 3; ++ks) {
      w0[0][ks] = blk0 >= 0 ? L.ws_a0[(blk0 * 3 + ks) * 64 + lane] : 0.f;
      w0[1][ks] = blk1 >= 0 ? L.ws_a0[(blk1 * 3 + ks) * 64 + lane] : 0.f;
    }
    const frag_t* WA = (const frag_t*)L.ws_ah;
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) w[rb][ks] = WA[(((team * 4 + tw) * 2 + rb) * 16 + ks) * 64 + lane];
    // wait here for every weight (vmcnt 0): otherwise the first uses inside the
    // stage loop carry waits that also cover the control wave's prefetches
    __builtin_amdgcn_s_waitcnt(0x0F70);
  }
};

__device__ inline void pipe_store4(uint16_t* dst, uint16_t h0, uint16_t h1, uint16_t h2, uint16_t h3) {
  uint2 packed;
  packed.x = (uint32_t)h0 | ((uint32_t)h1 << 16);
  packed.y = (uint32_t)h2 | ((uint32_t)h3 << 16);
  *(uint2*)dst = packed;
}

// First sine layer, rows [32 blk, 32 blk + 32) of one tile (operand W.w0[slot]).
template <int C, int P, bool TAN>
__device__ inline void pipe_layer0(const PipeWeights<P>& W, int slot, const float4* xin, uint16_t* dst, int d_in, int blk,
                                   const PipeLane& pl) {
  const int ks0 = d_in == 4 ? 3 : 2;
#pragma unroll
  for (int cb = 0; cb < (C / 32); ++cb) {
    const int col = 32 * cb + pl.j;
    const float4 in = xin[col];
    f32x16_t acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.f;
#pragma unroll
    for (int ks = 0; ks < 3; ++ks)
      if (ks < ks0)
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(W.w0[slot][ks], layer0_input(in, d_in, pl.c, ks, pl.g), acc, 0, 0, 0);
#pragma unroll
    for (int b4 = 0; b4 < 4; ++b4) {
      uint16_t h[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) h[i] = PipeBits<P>::bits(pipe_act<TAN, true>(acc[4 * b4 + i], pl));
      pipe_store4(&dst[col * kPipeStride + 32 * blk + 8 * b4 + 4 * pl.g], h[0], h[1], h[2], h[3]);
    }
  }
}

// Hidden product of one team wave: acc = bias + W[rows] act (the caller passes
// a zero bias for tangent columns).
template <int C, int P>
__device__ inline void pipe_hidden(const PipeWeights<P>& W, const uint16_t* src, const float* bias,
                                   f32x16_t (&acc)[(C / 32)][2], int tw, const PipeLane& pl) {
  typedef HiddenOps<P> Ops;
  typedef typename Ops::frag_t frag_t;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int b4 = 0; b4 < 4; ++b4) {
      const float4 b = *(const float4*)&bias[64 * tw + 32 * rb + 8 * b4 + 4 * pl.g];
#pragma unroll
      for (int cb = 0; cb < (C / 32); ++cb) {
        acc[cb][rb][4 * b4 + 0] = b.x;
        acc[cb][rb][4 * b4 + 1] = b.y;
        acc[cb][rb][4 * b4 + 2] = b.z;
        acc[cb][rb][4 * b4 + 3] = b.w;
      }
    }
#pragma unroll
  for (int ks = 0; ks < 16; ++ks) {
    frag_t b[(C / 32)];
#pragma unroll
    for (int cb = 0; cb < (C / 32); ++cb)
      b[cb] = *(const frag_t*)&src[(32 * cb + pl.j) * kPipeStride + 16 * ks + 8 * pl.g];
#pragma unroll
    for (int cb = 0; cb < (C / 32); ++cb)
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) acc[cb][rb] = Ops::mfma(W.w[rb][ks], b[cb], acc[cb][rb]);
  }
}

// The hidden product of a team-1 wave that also computes one of the control
// wave's W_1 row blocks (A from LDS): three accumulator chains (the wave's two
// row blocks and the LDS block) in one k loop share each B fragment and keep
// the matrix pipe busy while the LDS operands arrive; same k order as
// pipe_hidden.
template <int C, int P>
__device__ inline void pipe_hidden3(const PipeWeights<P>& W, const uint4* wlds, int blk, const uint16_t* src,
                                    const float* bias, f32x16_t (&acc)[(C / 32)][2], f32x16_t (&acc1)[(C / 32)],
                                    int tw, const PipeLane& pl) {
  typedef HiddenOps<P> Ops;
  typedef typename Ops::frag_t frag_t;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int b4 = 0; b4 < 4; ++b4) {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      const float4 b = *(const float4*)&bias[64 * tw + 32 * rb + 8 * b4 + 4 * pl.g];
#pragma unroll
      for (int cb = 0; cb < (C / 32); ++cb) {
        acc[cb][rb][4 * b4 + 0] = b.x;
        acc[cb][rb][4 * b4 + 1] = b.y;
        acc[cb][rb][4 * b4 + 2] = b.z;
        acc[cb][rb][4 * b4 + 3] = b.w;
      }
    }
    const float4 b = *(const float4*)&bias[32 * blk + 8 * b4 + 4 * pl.g];
#pragma unroll
    for (int cb = 0; cb < (C / 32); ++cb) {
      acc1[cb][4 * b4 + 0] = b.x;
      acc1[cb][4 * b4 + 1] = b.y;
      acc1[cb][4 * b4 + 2] = b.z;
      acc1[cb][4 * b4 + 3] = b.w;
    }
  }
#pragma unroll
  for (int ks = 0; ks < 16; ++ks) {
    const frag_t a = *(const frag_t*)&wlds[(blk * 16 + ks) * 64 + lane];
    frag_t b[(C / 32)];
#pragma unroll
    for (int cb = 0; cb < (C / 32); ++cb)
      b[cb] = *(const frag_t*)&src[(32 * cb + pl.j) * kPipeStride + 16 * ks + 8 * pl.g];
#pragma unroll
    for (int cb = 0; cb < (C / 32); ++cb) {
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) acc[cb][rb] = Ops::mfma(W.w[rb][ks], b[cb], acc[cb][rb]);
      acc1[cb] = Ops::mfma(a, b[cb], acc1[cb]);
    }
  }
}

template <int C, int P, bool TAN, bool RED>
__device__ inline void pipe_store_blk(const f32x16_t (&acc)[(C / 32)], uint16_t* dst, int blk, const PipeLane& pl) {
#pragma unroll
  for (int cb = 0; cb < (C / 32); ++cb)
#pragma unroll
    for (int b4 = 0; b4 < 4; ++b4) {
      uint16_t h[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) h[i] = PipeBits<P>::bits(pipe_act<TAN, RED>(acc[cb][4 * b4 + i], pl));
      pipe_store4(&dst[(32 * cb + pl.j) * kPipeStride + 32 * blk + 8 * b4 + 4 * pl.g], h[0], h[1], h[2], h[3]);
    }
}

template <int C, int P, bool TAN, bool RED>
__device__ inline void pipe_store(const f32x16_t (&acc)[(C / 32)][2], uint16_t* dst, int tw, const PipeLane& pl) {
#pragma unroll
  for (int cb = 0; cb < (C / 32); ++cb)
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int b4 = 0; b4 < 4; ++b4) {
        uint16_t h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) h[i] = PipeBits<P>::bits(pipe_act<TAN, RED>(acc[cb][rb][4 * b4 + i], pl));
        pipe_store4(&dst[(32 * cb + pl.j) * kPipeStride + 64 * tw + 32 * rb + 8 * b4 + 4 * pl.g], h[0], h[1], h[2],
                    h[3]);
      }
}

// sin of a team-2 wave's rows, dotted with the output weights in float32.
// Four partial sums keep the fma chain short.
template <bool TAN, bool RED>
__device__ inline float pipe_dot(const f32x16_t (&acc)[2], const float* wk, int tw, const PipeLane& pl) {
  float s[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int b4 = 0; b4 < 4; ++b4) {
      const float4 w = *(const float4*)&wk[64 * tw + 32 * rb + 8 * b4 + 4 * pl.g];
      s[0] = fmaf(w.x, pipe_act<TAN, RED>(acc[rb][4 * b4 + 0], pl), s[0]);
      s[1] = fmaf(w.y, pipe_act<TAN, RED>(acc[rb][4 * b4 + 1], pl), s[1]);
      s[2] = fmaf(w.z, pipe_act<TAN, RED>(acc[rb][4 * b4 + 2], pl), s[2]);
      s[3] = fmaf(w.w, pipe_act<TAN, RED>(acc[rb][4 * b4 + 3], pl), s[3]);
    }
  const float t = (s[0] + s[1]) + (s[2] + s[3]);
  return half_sum(t);
}  // (one 32-column block; callers loop over the tile's blocks)

template <int C>
__device__ inline void pipe_setup(PipeSmem<C>& sm, const DevLevel& L) {
  for (int i = threadIdx.x; i < 256; i += kPipeThreads) {
    sm.bias[0][i] = L.bh_plain[i];
    sm.bias[1][i] = L.bh_plain[256 + i];
    sm.wk[i] = L.wk_plain[i];
    sm.zeros[i] = 0.f;
  }
  for (int i = threadIdx.x; i < kPipeGroups * C; i += kPipeThreads)
    sm.srec[i / C][2][i % C] = make_float4(__int_as_float(-1), 0.f, 0.f, 0.f);
  if (threadIdx.x < 8) sm.tlive[threadIdx.x] = 0;
  if (threadIdx.x < 2) sm.stop[threadIdx.x] = 0;
  if (threadIdx.x < 4) sm.simd_count[threadIdx.x] = 0;
  if constexpr (C == 32 && NNM_WS_CTL_NOH1) {
    // team 1, wave 0, row blocks 0 and 1 of W_1: the first 2 x 16 x 64 fragments of ws_ah
    const uint4* src = (const uint4*)L.ws_ah;
    for (int i = threadIdx.x; i < 2 * 16 * 64; i += kPipeThreads) sm.w1lds[i] = src[i];
  }
}

// Role of this wave, 4 team + simd: the first wave that arrives on a SIMD joins
// team 1, the second team 2, so every SIMD pairs one wave of each team whatever
// placement the dispatcher chose.  (Eight waves of 256 registers fill the four
// register files exactly, so each SIMD holds two of them; if the counts say
// otherwise the wave index decides.)  Contains a workgroup barrier.
template <int C>
__device__ inline int pipe_role(PipeSmem<C>& sm) {
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    // HW_ID bits [5:4]: the SIMD this wave runs on
    const int simd = (__builtin_amdgcn_s_getreg((1 << 11) | (4 << 6) | 4)) & 3;
    const int slot = atomicAdd(&sm.simd_count[simd], 1);
    sm.role_of[wave] = 4 * slot + simd;
  }
  __syncthreads();
  const bool paired = sm.simd_count[0] == 2 && sm.simd_count[1] == 2 && sm.simd_count[2] == 2 && sm.simd_count[3] == 2;
  return __builtin_amdgcn_readfirstlane(paired ? sm.role_of[wave] : wave);
}

// Stage s of the evaluating roles.  Team 1: the first hidden product of tile
// s-1 and its sines, then its block of the first layer of tile s (role 0 runs
// the control in between).  Team 2 in two calls: the output sines of tile s-3,
// then its first-layer block of tile s and the second hidden product of tile
// s-2, whose accumulators carry into stage s+1.
template <int C, int P, bool TAN, bool RED>
__device__ inline void pipe_team1_hidden(PipeSmem<C>& sm, const PipeWeights<P>& W, f32x16_t (&acc)[(C / 32)][2], int s,
                                         int wave, const PipeLane& pl) {
  if (sm.tlive[(s + 7) & 7]) {
    constexpr bool kNoH1 = C == 32 && !TAN && NNM_WS_CTL_NOH1;
    if (kNoH1 && wave == 0) return;
    if (kNoH1 && (wave == 1 || wave == 2)) {
      f32x16_t acc1[(C / 32)];
      pipe_hidden3<C, P>(W, sm.w1lds, wave - 1, sm.act0[(s + 1) & 1], sm.bias[0], acc, acc1, wave & 3, pl);
      pipe_store<C, P, TAN, RED>(acc, sm.act1[(s + 1) & 1], wave & 3, pl);
      pipe_store_blk<C, P, TAN, RED>(acc1, sm.act1[(s + 1) & 1], wave - 1, pl);
      return;
    }
    pipe_hidden<C, P>(W, sm.act0[(s + 1) & 1], (TAN && pl.c) ? sm.zeros : sm.bias[0], acc, wave & 3, pl);
    pipe_store<C, P, TAN, RED>(acc, sm.act1[(s + 1) & 1], wave & 3, pl);
  }
}

// OFF0: role 0 (the control wave) hands its first-layer block to role 1.
template <int C, int P, bool TAN, bool OFF0>
__device__ inline void pipe_team1_layer0(PipeSmem<C>& sm, const PipeWeights<P>& W, const DevLevel& L, int s, int wave,
                                         const PipeLane& pl) {
  if (!sm.tlive[s & 7]) return;
  if (!OFF0 || wave != 0) pipe_layer0<C, P, TAN>(W, 0, sm.xin[s & 1], sm.act0[s & 1], L.d_in, wave, pl);
  if (OFF0 && wave == kOff0Wave) pipe_layer0<C, P, TAN>(W, 1, sm.xin[s & 1], sm.act0[s & 1], L.d_in, 0, pl);
}

#ifndef NNM_NORMAL_L0_MODE
#define NNM_NORMAL_L0_MODE 1
#endif
// First-layer row blocks (0..7, 32 rows each) of the normal kernel per role,
// -1 for none.  Its team-2 waves carry the sines and output dot products of
// four columns per point and set the stage time, so roles 5-7 compute no
// first-layer block; roles 1-3 compute blocks w and w + 4.  Mode 0 is the
// tracing kernel's assignment (one block per wave, role 1 taking the control
// wave's); modes 2 and 3 move block 4 to role 0 or block 0 to role 4.
__device__ inline int normal_blk(int wave, int slot) {
  constexpr int mode = NNM_NORMAL_L0_MODE;
  if (mode == 0) return slot == 0 ? (wave == 0 ? -1 : wave) : (wave == 1 ? 0 : -1);
  if (wave >= 1 && wave <= 3) return slot == 0 ? wave : wave + 4;
  if (wave == 0) return slot == 0 ? (mode == 3 ? -1 : 0) : (mode == 2 ? 4 : -1);
  if (wave == 4) return slot == 0 ? (mode == 2 ? -1 : 4) : (mode == 3 ? 0 : -1);
  return -1;
}

template <int C, int P>
__device__ inline void pipe_normal_layer0(PipeSmem<C>& sm, const PipeWeights<P>& W, const DevLevel& L, int s, int wave,
                                          const PipeLane& pl) {
  if (!sm.tlive[s & 7]) return;
  const int b0 = normal_blk(wave, 0), b1 = normal_blk(wave, 1);
  if (b0 >= 0) pipe_layer0<C, P, true>(W, 0, sm.xin[s & 1], sm.act0[s & 1], L.d_in, b0, pl);
  if (b1 >= 0) pipe_layer0<C, P, true>(W, 1, sm.xin[s & 1], sm.act0[s & 1], L.d_in, b1, pl);
}

template <int C, bool TAN, bool RED>
__device__ inline void pipe_team2_out(PipeSmem<C>& sm, const f32x16_t (&acc)[(C / 32)][2], int s, int wave,
                                      const PipeLane& pl) {
  const int tw = wave & 3;
  if (sm.tlive[(s + 5) & 7]) {
#pragma unroll
    for (int cb = 0; cb < (C / 32); ++cb) {
      const float p = pipe_dot<TAN, RED>(acc[cb], sm.wk, tw, pl);
      if (pl.g == 0) sm.part[(s + 1) & 1][tw][32 * cb + pl.j] = p;
    }
  }
}

// L0: this call computes the wave's first-layer block (the normal kernel does
// its first layer in pipe_normal_layer0 instead).
template <int C, int P, bool TAN, bool L0 = true>
__device__ inline void pipe_team2_in(PipeSmem<C>& sm, const PipeWeights<P>& W, const DevLevel& L,
                                     f32x16_t (&acc)[(C / 32)][2], int s, int wave, const PipeLane& pl) {
  const int tw = wave & 3;
  if (L0 && sm.tlive[s & 7]) pipe_layer0<C, P, TAN>(W, 0, sm.xin[s & 1], sm.act0[s & 1], L.d_in, wave, pl);
  if (sm.tlive[(s + 6) & 7]) {
    pipe_hidden<C, P>(W, sm.act1[s & 1], (TAN && pl.c) ? sm.zeros : sm.bias[1], acc, tw, pl);
  } else {
    // overwritten on both paths: the accumulators are dead between the two calls
#pragma unroll
    for (int cb = 0; cb < (C / 32); ++cb)
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[cb][rb][r] = 0.f;
  }
}

// Tile liveness and the stop flag, written by lane 0 of the control wave;
// glive is the control wave's bitmask of groups holding rays.
template <int C>
__device__ inline void pipe_publish(PipeSmem<C>& sm, int s, int glive, bool live, bool more) {
  sm.tlive[(s + 1) & 7] = live ? 1 : 0;
  sm.stop[(s + 2) & 1] = (glive == 0 && !more) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Tracing control (role 0): 64 ray slots per group, one per lane, and a
// 64-entry staging ring of prefetched rays (lane e holds entry e) that refills
// freed slots by lane shuffles and is topped up right after, so its loads
// complete while the pipeline runs.
struct TraceCtl {
  int s_ray, s_st;
  float s_ox, s_oy, s_oz, s_vx, s_vy, s_vz, s_tt, s_tau;
  int s_head, s_count;
  int cur, end, seg, chunk, n_in;
  bool exhausted;
  PushRing pr;
  int glive;  // bit G: slot group G holds rays
  int park_head, park_count;

  __device__ inline void init(PipeSmem<kTraceCols>& sm, const TraceLevelArgs& A, int lane) {
    glive = 0;
    park_head = park_count = 0;
    n_in = A.in_count ? *A.in_count : A.n;
    s_ray = -1;
    s_st = 0;
    s_ox = s_oy = s_oz = s_vx = s_vy = s_vz = s_tt = s_tau = 0.f;
    s_head = s_count = 0;
    cur = end = 0;
#ifndef NNM_WS_CHUNK_DIV
#define NNM_WS_CHUNK_DIV 8
#endif
    chunk = min(kChunk, max(64, (n_in / (NNM_WS_CHUNK_DIV * (int)gridDim.x)) & ~63));
    seg = blockIdx.x % kSegments;
    exhausted = false;
    sm.hist[lane] = 0;  // (only this wave touches it)
  }

  // Fill the staging ring up to 64 entries from the segmented input queue.
  __device__ inline void top_up(const TraceLevelArgs& A, int lane) {
    while (s_count < 64 && !exhausted) {
      if (cur >= end) {
        int s0, s_len;
        segment_bounds(seg, n_in, s0, s_len);
        int base = 0;
        if (lane == 0) base = atomicAdd(A.in_heads + seg * kHeadStride, chunk);
        base = __shfl(base, 0);
        if (base >= s_len) {
          // this segment is drained: on to one that is not, if any
          seg = next_open_segment(A.in_heads, n_in, blockIdx.x, lane);
          if (seg < 0) exhausted = true;
          continue;
        }
        cur = s0 + base;
        end = s0 + min(base + chunk, s_len);
      }
      const int add = min(64 - s_count, end - cur);
      const int q = ((lane - s_head) & 63) - s_count;
      if (q >= 0 && q < add) {
        const int idx = cur + q;
        s_ray = A.in_queue ? A.in_queue[idx] : idx;
        s_ox = A.o[3 * s_ray + 0];
        s_oy = A.o[3 * s_ray + 1];
        s_oz = A.o[3 * s_ray + 2];
        s_vx = A.v[3 * s_ray + 0];
        s_vy = A.v[3 * s_ray + 1];
        s_vz = A.v[3 * s_ray + 2];
        s_tt = A.t ? A.t[s_ray] : 0.f;
        if (A.level == 0) {
          s_tau = 0.f;
          s_st = 0;
          if (A.steps)
            for (int jj = 1; jj < A.m; ++jj) A.steps[(long long)s_ray * A.m + jj] = 0;
        } else {
          s_tau = A.depth[s_ray];
          s_st = A.status[s_ray];
        }
      }
      s_count += add;
      cur += add;
    }
  }

  // Rays that left the level (to the next level or the normal pass), with
  // their order keys when the next level's queue is sorted.
  __device__ inline void push(PipeSmem<kTraceCols>& sm, const TraceLevelArgs& A, int lane, bool done, int ray, int k) {
    if (!A.out_queue) return;
    const unsigned long long pm = __ballot(done);
    if (!pm) return;
    uint8_t* rk = A.out_key ? sm.ring_key : nullptr;
    pr.add(sm.ring, rk, pm, done, __popcll(pm & ((1ull << lane) - 1ull)), ray, order_key(k));
    if (pr.n >= kPushBatch) pr.publish(sm.ring, rk, lane, A.out_count, A.out_queue, A.out_key, sm.hist, false);
  }

  __device__ inline void flush(PipeSmem<kTraceCols>& sm, const TraceLevelArgs& A, int lane) {
    if (!A.out_queue) return;
    uint8_t* rk = A.out_key ? sm.ring_key : nullptr;
    if (pr.n > 0) pr.publish(sm.ring, rk, lane, A.out_count, A.out_queue, A.out_key, sm.hist, true);
    if (A.out_key) {
      const int c = sm.hist[lane];
      if (c) atomicAdd(A.out_hist + lane, c);
    }
  }

  // Stage s (s = -1: prologue): finish tile s-4, refill its group, write tile s+1.
  __device__ inline void step(PipeSmem<kTraceCols>& sm, const TraceLevelArgs& A, int s, int lane) {
    const DevLevel& L = A.L;
    const int G = (s + 1) % kPipeGroups;
    const bool slot = lane < kTraceCols;
    const int sl = lane & (kTraceCols - 1);
    int ray = -1, k = 0, st = 0;
    float tau = 0.f, ox = 0.f, oy = 0.f, oz = 0.f, vx = 0.f, vy = 0.f, vz = 0.f, tt = 0.f, cx = 0.f, cy = 0.f;
    if (slot) {
      const float4 r0 = sm.srec[G][0][sl], r1 = sm.srec[G][1][sl], r2 = sm.srec[G][2][sl];
      ox = r0.x;
      oy = r0.y;
      oz = r0.z;
      tau = r0.w;
      vx = r1.x;
      vy = r1.y;
      vz = r1.z;
      tt = r1.w;
      ray = __float_as_int(r2.x);
      k = __float_as_int(r2.y) & 0xFFFF;
      st = __float_as_int(r2.y) >> 16;
      cx = r2.z;
      cy = r2.w;
    }
    // Algorithm 1 update with the outputs of tile s-4 (part[(s - 4) % 2])
    int outcome = 0;
    if (ray >= 0) {
      const int pb = s & 1;
      const float N = sm.part[pb][0][sl] + sm.part[pb][1][sl] + sm.part[pb][2][sl] + sm.part[pb][3][sl] + L.bk;
      float base_term = 0.f;
      if (A.B.sphere) {
        const float x = fmaf(tau, vx, ox), y = fmaf(tau, vy, oy), z = fmaf(tau, vz, oz);
        const float dx = x - cx, dy = y - cy;
        base_term = base_radius(dx, dy, z) - A.B.r0;
      }
      const float f = fmaf(L.amplitude, N, base_term);
      outcome = alg1_step(A, f - A.delta, tau, k, st);
    }
    push(sm, A, lane, outcome == 1, ray, k);
    if (outcome != 0) {
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
      ray = -1;
    }
    // Tail compaction.  Once the queue is drained, a group with few survivors
    // parks them in LDS and its next tile is dark (a cheap stage); the next
    // group with free slots takes them in.  Live rays so gather in fewer tiles
    // while the last, longest rays finish.
    bool parked = false;
    if (exhausted && s_count == 0 && park_count == 0) {
      const unsigned long long smask = __ballot(slot && ray >= 0);
      const int nsurv = __popcll(smask);
      if (nsurv > 0 && nsurv <= kParkMax) {
        if (slot && ray >= 0) {
          const int e = (park_head + __popcll(smask & ((1ull << lane) - 1ull))) & (kTraceCols - 1);
          sm.park[0][e] = make_float4(ox, oy, oz, tau);
          sm.park[1][e] = make_float4(vx, vy, vz, tt);
          sm.park[2][e] = make_float4(__int_as_float(ray), __int_as_float(k | (st << 16)), cx, cy);
          ray = -1;
        }
        park_count = nsurv;
        parked = true;
      }
    }
    // refill freed slots: parked rays first, then the staging ring
    if (!parked && park_count > 0) {
      const unsigned long long fmask = __ballot(slot && ray < 0);
      const int takep = min((int)__popcll(fmask), park_count);
      const int p = __popcll(fmask & ((1ull << lane) - 1ull));
      if (slot && ray < 0 && p < takep) {
        const int e = (park_head + p) & (kTraceCols - 1);
        const float4 r0 = sm.park[0][e], r1 = sm.park[1][e], r2 = sm.park[2][e];
        ox = r0.x;
        oy = r0.y;
        oz = r0.z;
        tau = r0.w;
        vx = r1.x;
        vy = r1.y;
        vz = r1.z;
        tt = r1.w;
        ray = __float_as_int(r2.x);
        k = __float_as_int(r2.y) & 0xFFFF;
        st = __float_as_int(r2.y) >> 16;
        cx = r2.z;
        cy = r2.w;
      }
      park_head = (park_head + takep) & (kTraceCols - 1);
      park_count -= takep;
    }
    const unsigned long long emask = __ballot(slot && ray < 0);
    const int take = min((int)__popcll(emask), s_count);
    const int p = __popcll(emask & ((1ull << lane) - 1ull));
    const bool fill = slot && ray < 0 && p < take;
    const int src = fill ? ((s_head + p) & 63) : lane;
    const int n_ray = __shfl(s_ray, src), n_st = __shfl(s_st, src);
    const float n_ox = __shfl(s_ox, src), n_oy = __shfl(s_oy, src), n_oz = __shfl(s_oz, src);
    const float n_vx = __shfl(s_vx, src), n_vy = __shfl(s_vy, src), n_vz = __shfl(s_vz, src);
    const float n_tt = __shfl(s_tt, src), n_tau = __shfl(s_tau, src);
    if (fill) {
      ray = n_ray;
      st = n_st;
      ox = n_ox;
      oy = n_oy;
      oz = n_oz;
      vx = n_vx;
      vy = n_vy;
      vz = n_vz;
      tt = n_tt;
      tau = n_tau;
      k = 0;
      center_at(A.B, tt, cx, cy);  // c(t) is fixed per ray: once, on entry
    }
    s_head = (s_head + take) & 63;
    s_count -= take;
    // top up in batches of at least 32 entries: the loop and its queue atomics
    // then run on a few stages only
    if (s_count <= 32) top_up(A, lane);
    // inputs of tile s+1
    const bool live = __ballot(slot && ray >= 0) != 0ull;
    if (slot) {
      sm.srec[G][0][sl] = make_float4(ox, oy, oz, tau);
      sm.srec[G][1][sl] = make_float4(vx, vy, vz, tt);
      sm.srec[G][2][sl] = make_float4(__int_as_float(ray), __int_as_float(k | (st << 16)), cx, cy);
      sm.xin[(s + 1) & 1][sl] = net_input(L, fmaf(tau, vx, ox), fmaf(tau, vy, oy), fmaf(tau, vz, oz), tt, cx, cy);
    }
    glive = live ? (glive | (1 << G)) : (glive & ~(1 << G));
    if (lane == 0) pipe_publish(sm, s, glive, live, s_count > 0 || !exhausted || park_count > 0);
  }
};

// One team's side of the tracing kernel; role 0 (team 1) runs the control and
// holds no weights (its W_1 rows are in LDS), so its loop is separate and the
// register budget of the evaluating roles does not include the control's
// state.  Every wave executes the same number of workgroup barriers.
template <int P, bool RED, bool TEAM2>
__device__ inline void trace_body(PipeSmem<kTraceCols>& sm, const TraceLevelArgs& A, int wave, int lane) {
  if (!TEAM2 && wave == 0 && NNM_WS_CTL_NOH1) {
    TraceCtl ctl;
    ctl.init(sm, A, lane);
    ctl.top_up(A, lane);
    __syncthreads();
    ctl.step(sm, A, -1, lane);
    __syncthreads();
    for (int s = 0;; ++s) {
      if (sm.stop[(s + 1) & 1]) break;
      ctl.step(sm, A, s, lane);
      __syncthreads();
    }
    ctl.flush(sm, A, lane);
    return;
  }
  PipeWeights<P> W;
  W.load(A.L, wave, lane, wave, wave == kOff0Wave ? 0 : -1);  // this role also computes the control wave's block
  const PipeLane pl = pipe_lane<false>(lane);
  const bool ctl_wave = !TEAM2 && wave == 0;
  TraceCtl ctl;
  if (ctl_wave) {
    ctl.init(sm, A, lane);
    ctl.top_up(A, lane);
  }
  __syncthreads();
  if (ctl_wave) ctl.step(sm, A, -1, lane);
  __syncthreads();
  f32x16_t acc[kTraceCols / 32][2];
  for (int s = 0;; ++s) {
    if (sm.stop[(s + 1) & 1]) break;
    if (!TEAM2) {
      pipe_team1_hidden<kTraceCols, P, false, RED>(sm, W, acc, s, wave, pl);
      if (ctl_wave) ctl.step(sm, A, s, lane);
      pipe_team1_layer0<kTraceCols, P, false, true>(sm, W, A.L, s, wave, pl);
    } else {
      pipe_team2_out<kTraceCols, false, RED>(sm, acc, s, wave, pl);
      pipe_team2_in<kTraceCols, P, false>(sm, W, A.L, acc, s, wave, pl);
    }
    __syncthreads();
  }
  if (ctl_wave) ctl.flush(sm, A, lane);
}

template <int P, bool RED>
__global__ void __launch_bounds__(kPipeThreads, 1) k_trace_ws(TraceLevelArgs A) {
  __shared__ PipeSmem<kTraceCols> sm;
  pipe_setup(sm, A.L);
  __syncthreads();
  const int wave = pipe_role(sm);
  if (wave < 4)
    trace_body<P, RED, false>(sm, A, wave, threadIdx.x & 63);
  else
    trace_body<P, RED, true>(sm, A, wave, threadIdx.x & 63);
}

// ---------------------------------------------------------------------------
// Normal control (role 0): 16 points per group (columns 4 q + c), fetched ahead:
// in stage s the ray data of tile s+2 and the queue entries of tile s+3 are
// loaded, so no stage waits on memory.
struct NormalCtl {
  int n_in, next;  // next: first queue slot of the next tile this workgroup fetches
  int q_ray;       // lanes 0..15: queue entries two tiles ahead
  int p_ray;       // lanes 0..15: rays of the next tile, with their data
  float p_ox, p_oy, p_oz, p_vx, p_vy, p_vz, p_tau, p_t;
  int glive;  // bit G: slot group G holds points

  __device__ inline int fetch_id(const NormalArgs& A, int lane) {
    const int slot = next + lane;
    const int r = (lane < (kNormalCols / 4) && slot < n_in) ? (A.queue ? A.queue[slot] : slot) : -1;
    next += (kNormalCols / 4) * gridDim.x;
    return r;
  }
  __device__ inline void fetch_data(const NormalArgs& A) {
    if (p_ray >= 0) {
      if (A.x) {
        // points mode: tau = 0 and v = 0 make the end point x itself
        p_ox = A.x[3 * p_ray + 0];
        p_oy = A.x[3 * p_ray + 1];
        p_oz = A.x[3 * p_ray + 2];
        p_vx = p_vy = p_vz = p_tau = 0.f;
      } else {
        p_ox = A.o[3 * p_ray + 0];
        p_oy = A.o[3 * p_ray + 1];
        p_oz = A.o[3 * p_ray + 2];
        p_vx = A.v[3 * p_ray + 0];
        p_vy = A.v[3 * p_ray + 1];
        p_vz = A.v[3 * p_ray + 2];
        p_tau = A.depth[p_ray];
      }
      p_t = A.t ? A.t[p_ray] : 0.f;
    }
  }
  __device__ inline void init(const NormalArgs& A, int lane) {
    n_in = A.count ? *A.count : A.n;
    next = blockIdx.x * (kNormalCols / 4);
    glive = 0;
    p_ox = p_oy = p_oz = p_vx = p_vy = p_vz = p_tau = p_t = 0.f;
    p_ray = fetch_id(A, lane);
    fetch_data(A);
    q_ray = fetch_id(A, lane);
  }

  __device__ inline void step(PipeSmem<kNormalCols>& sm, const NormalArgs& A, int s, int lane) {
    const DevLevel& L = A.L;
    const int G = (s + 1) % kPipeGroups;
    const bool col = lane < kNormalCols;
    const int q = (lane >> 2) & ((kNormalCols / 4) - 1), c = lane & 3;
    // normals of tile s-4
    if (glive & (1 << G)) {
      const int pb = s & 1;
      const int sl = lane & (kNormalCols - 1);
      float val = sm.part[pb][0][sl] + sm.part[pb][1][sl] + sm.part[pb][2][sl] + sm.part[pb][3][sl];
      if (c == 0) val += L.bk;
      const float gx = quad_bcast<1>(val), gy = quad_bcast<2>(val), gz = quad_bcast<3>(val);
      const int ray = __float_as_int(sm.srec[G][2][q].x);
      if (col && c == 0 && ray >= 0) {
        const float4 r0 = sm.srec[G][0][q], r1 = sm.srec[G][1][q];
        const float x = r0.x, y = r0.y, z = r0.z, cx = r1.x, cy = r1.y;
        float fx = L.amplitude * gx, fy = L.amplitude * gy, fz = L.amplitude * gz;
        if (A.B.sphere) {
          const float dx = x - cx, dy = y - cy;
          const float r2 = fmaf(dx, dx, fmaf(dy, dy, z * z));
          if (r2 > 0.f) {
            const float ir = rsqrtf(r2);
            fx = fmaf(dx, ir, fx);
            fy = fmaf(dy, ir, fy);
            fz = fmaf(z, ir, fz);
          }
        }
        const float len2 = fmaf(fx, fx, fmaf(fy, fy, fz * fz));
        const float inv = len2 > 0.f ? rsqrtf(len2) : 0.f;
        A.normal[3 * ray + 0] = fx * inv;
        A.normal[3 * ray + 1] = fy * inv;
        A.normal[3 * ray + 2] = fz * inv;
      }
    }
    // tile s+1 from the prefetched points (lanes 0..15)
    float x = 0.f, y = 0.f, z = 0.f, cx = 0.f, cy = 0.f;
    if (p_ray >= 0) {
      x = fmaf(p_tau, p_vx, p_ox);
      y = fmaf(p_tau, p_vy, p_oy);
      z = fmaf(p_tau, p_vz, p_oz);
      center_at(A.B, p_t, cx, cy);
    }
    const bool live = __ballot(p_ray >= 0) != 0ull;
    if (lane < (kNormalCols / 4)) {
      sm.srec[G][0][lane] = make_float4(x, y, z, 0.f);
      sm.srec[G][1][lane] = make_float4(cx, cy, 0.f, 0.f);
      sm.srec[G][2][lane] = make_float4(__int_as_float(p_ray), 0.f, 0.f, 0.f);
    }
    const float qx = __shfl(x, q), qy = __shfl(y, q), qz = __shfl(z, q), qt = __shfl(p_t, q);
    const float qcx = __shfl(cx, q), qcy = __shfl(cy, q);
    if (col) sm.xin[(s + 1) & 1][lane] = net_input(L, qx, qy, qz, qt, qcx, qcy);
    // prefetch: data of tile s+2, queue entries of tile s+3
    p_ray = q_ray;
    fetch_data(A);
    q_ray = fetch_id(A, lane);
    // later tiles hold points only if tile s+2 does (tiles are fetched in slot order)
    const bool more = __ballot(p_ray >= 0) != 0ull;
    glive = live ? (glive | (1 << G)) : (glive & ~(1 << G));
    if (lane == 0) pipe_publish(sm, s, glive, live, more);
  }
};

template <int P, bool RED, bool TEAM2>
__device__ inline void normal_body(PipeSmem<kNormalCols>& sm, const NormalArgs& A, int wave, int lane) {
  PipeWeights<P> W;
  W.load(A.L, wave, lane, normal_blk(wave, 0), normal_blk(wave, 1));
  const PipeLane pl = pipe_lane<true>(lane);
  const bool ctl_wave = !TEAM2 && wave == 0;
  NormalCtl ctl;
  if (ctl_wave) ctl.init(A, lane);
  __syncthreads();
  if (ctl_wave) ctl.step(sm, A, -1, lane);
  __syncthreads();
  f32x16_t acc[kNormalCols / 32][2];
  for (int s = 0;; ++s) {
    if (sm.stop[(s + 1) & 1]) break;
    if (!TEAM2) {
      pipe_team1_hidden<kNormalCols, P, true, RED>(sm, W, acc, s, wave, pl);
      if (ctl_wave) ctl.step(sm, A, s, lane);
      pipe_normal_layer0<kNormalCols, P>(sm, W, A.L, s, wave, pl);
    } else {
      pipe_team2_out<kNormalCols, true, RED>(sm, acc, s, wave, pl);
      pipe_normal_layer0<kNormalCols, P>(sm, W, A.L, s, wave, pl);
      pipe_team2_in<kNormalCols, P, true, false>(sm, W, A.L, acc, s, wave, pl);
    }
    __syncthreads();
  }
}

template <int P, bool RED>
__global__ void __launch_bounds__(kPipeThreads, 1) k_normal_ws(NormalArgs A) {
  __shared__ PipeSmem<kNormalCols> sm;
  pipe_setup(sm, A.L);
  __syncthreads();
  const int wave = pipe_role(sm);
  if (wave < 4)
    normal_body<P, RED, false>(sm, A, wave, threadIdx.x & 63);
  else
    normal_body<P, RED, true>(sm, A, wave, threadIdx.x & 63);
}

template <bool RED>
static hipError_t launch_trace_ws_r(int prec, const TraceLevelArgs& a, int grid, hipStream_t s) {
  if (prec == PREC_BF16)
    hipLaunchKernelGGL((k_trace_ws<PREC_BF16, RED>), dim3(grid), dim3(kPipeThreads), 0, s, a);
  else if (prec == PREC_FP16)
    hipLaunchKernelGGL((k_trace_ws<PREC_FP16, RED>), dim3(grid), dim3(kPipeThreads), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <bool RED>
static hipError_t launch_normal_ws_r(int prec, const NormalArgs& a, int grid, hipStream_t s) {
  if (prec == PREC_BF16)
    hipLaunchKernelGGL((k_normal_ws<PREC_BF16, RED>), dim3(grid), dim3(kPipeThreads), 0, s, a);
  else if (prec == PREC_FP16)
    hipLaunchKernelGGL((k_normal_ws<PREC_FP16, RED>), dim3(grid), dim3(kPipeThreads), 0, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_trace_ws(int prec, const TraceLevelArgs& a, int grid, hipStream_t s) {
  return a.L.reduce_hidden ? launch_trace_ws_r<true>(prec, a, grid, s) : launch_trace_ws_r<false>(prec, a, grid, s);
}

hipError_t launch_normal_ws(int prec, const NormalArgs& a, int grid, hipStream_t s) {
  return a.L.reduce_hidden ? launch_normal_ws_r<true>(prec, a, grid, s) : launch_normal_ws_r<false>(prec, a, grid, s);
}

int ws_resident_blocks(int prec, int kind, int device) {
  const void* fn = prec == PREC_FP16
                       ? (kind == 0 ? (const void*)k_trace_ws<PREC_FP16, false> : (const void*)k_normal_ws<PREC_FP16, false>)
                       : (kind == 0 ? (const void*)k_trace_ws<PREC_BF16, false> : (const void*)k_normal_ws<PREC_BF16, false>);
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kPipeThreads, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
  return per_cu * cus;
}

}  // namespace nnm

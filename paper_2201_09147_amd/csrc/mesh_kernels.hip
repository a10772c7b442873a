// mesh_kernels.hip -- the coarse triangle mesh that neural normal mapping
// decorates (Sec. 5, triangle-mesh example; Fig. 5 extracts it from a (64,1)
// network): scene-function values on a regular grid, then marching tetrahedra.
//
// Extraction reading (the paper uses marching cubes without fixing a variant):
// marching tetrahedra on the Kuhn subdivision of every grid cube, which gives a
// closed, consistently oriented piecewise-linear surface without case tables.
// The output order is fixed so that results do not depend on scheduling:
//   * a node is inside when value < iso (NaN is outside);
//   * each node owns seven edges, to node + D for D in the order
//     (1,0,0) (0,1,0) (0,0,1) (1,1,0) (1,0,1) (0,1,1) (1,1,1); an edge whose ends
//     differ carries one vertex at the zero of the linear interpolant, and
//     vertices are numbered in (node, edge) order;
//   * cube (i, j, k) holds six tetrahedra, one per axis order (a, b, c) in
//     lexicographic order, with corners 0, e_a, e_a + e_b, (1,1,1) and the middle
//     two swapped for odd orders (all positively oriented); triangles follow cube
//     order, then tetrahedron order;
//   * a tetrahedron (q0 q1 q2 q3) with one corner a alone on its side gives one
//     triangle on the edges from a to the others, taken in increasing order with
//     the last two swapped when a is odd (reversed when a is the outside one);
//     two inside corners a < b against c < d (c, d swapped for {0,2} and {1,3})
//     give (E(a,c), E(a,d), E(b,d)) and (E(a,c), E(b,d), E(b,c)).  Every triangle
//     then faces from the inside to the outside.
//
// Six launches: corner bytes, per-workgroup vertex and triangle counts, a
// two-level exclusive scan of those counts, vertex emission (a surface node
// records its first vertex id) and triangle emission (which reads the vertex
// ids of the neighbouring nodes).  Only the first pass reads the grid values
// in full.
#include "trace_common.h"

namespace nnm {

// ------------------------------------------------------------ grid values

__device__ inline float grid_coord(float lo, float hi, int res, int i) {
  return (float)((double)lo + ((double)hi - (double)lo) * (double)i / (double)(res - 1));
}

template <int H, int P>
__global__ void __launch_bounds__(kBlockThreads) k_grid_values(GridArgs A) {
  __shared__ NetSmem<H> sm;
  stage_net<H>(&sm, A.L);
  const int lane = threadIdx.x & 63;
  const int col = lane & 31;
  const int g = lane >> 5;
  const int wave = blockIdx.x * (kBlockThreads / 64) + (threadIdx.x >> 6);
  const int nwaves = gridDim.x * (kBlockThreads / 64);
  SirenTile<H, P, false> tile;
  float cx, cy;
  center_at(A.B, A.t, cx, cy);
  for (int base = wave * 32; base < A.n; base += nwaves * 32) {
    const int node = base + col;
    const bool live = node < A.n;
    float x = 0.f, y = 0.f, z = 0.f;
    if (live) {
      const int i = node % A.res, j = (node / A.res) % A.res, k = node / (A.res * A.res);
      x = grid_coord(A.lo, A.hi, A.res, i);
      y = grid_coord(A.lo, A.hi, A.res, j);
      z = grid_coord(A.lo, A.hi, A.res, k);
    }
    const float N = tile.eval(&sm, A.L, net_input(A.L, x, y, z, A.t, cx, cy), 0);
    if (g == 0 && live) {
      float base_term = 0.f;
      if (A.B.sphere) {
        const float dx = x - cx, dy = y - cy;
        base_term = sqrtf(fmaf(dx, dx, fmaf(dy, dy, z * z))) - A.B.r0;
      }
      A.values[node] = fmaf(A.L.amplitude, N, base_term);
    }
  }
}

static int occupancy_blocks(const void* fn, int threads, int device) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0) != hipSuccess || per_cu < 1) per_cu = 1;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus < 1) cus = 1;
  return per_cu * cus;
}

hipError_t launch_grid_values(int width, int prec, const GridArgs& a, int device, hipStream_t s) {
  const long long want = ((long long)a.n + 127) / 128;  // 32 nodes per wave, 4 waves
#define CALL(H, P)                                                                             \
  {                                                                                            \
    const int resident = occupancy_blocks((const void*)k_grid_values<H, P>, kBlockThreads, device); \
    const int grid = (int)std::max(1LL, std::min(want, 4LL * resident));                     \
    hipLaunchKernelGGL((k_grid_values<H, P>), dim3(grid), dim3(kBlockThreads), 0, s, a);     \
  }
  NNM_DISPATCH(width, prec, CALL)
#undef CALL
  return hipGetLastError();
}

// ------------------------------------------------------- marching tetrahedra
//
// Pass 1 (k_mt_mask) stores one byte per node: bit c is the inside bit of
// corner c of the node's cube (bit 0 = +x, bit 1 = +y, bit 2 = +z), corners
// outside the grid copying corner 0 so that they never look like a crossing.
// A wave owns 64 consecutive x of kMaskRows rows of one slice: its loads are
// coalesced rows, the x + 1 neighbours come from a ballot, and each row is
// loaded once for the two node rows that use it.
//
// The other passes walk the nodes in their linear order in flat runs of kFlat
// nodes per thread (one 16-byte load of corner bytes), so that workgroups and
// threads own increasing, contiguous node ranges and one workgroup scan of
// per-thread counts gives node-ordered vertex and triangle ids.  Workgroups
// without a surface node leave after one vote.  Triangle emission gathers the
// corner bytes and first vertex ids of the cube's seven lower corners in one
// round trip and derives the ids of all nineteen Kuhn edges from them.

constexpr int kMaskRows = 8;  // node rows per wave in the corner-byte pass
constexpr int kFlat = 16;     // nodes per thread in the counting and emission passes

// Edge direction d (order above) as a corner code, and back.
__host__ __device__ constexpr int dir_code(int d) {
  return d < 3 ? (1 << d) : (d == 3 ? 3 : (d == 4 ? 5 : (d == 5 ? 6 : 7)));
}
__host__ __device__ constexpr int code_dir(int code) {
  // 1 -> 0, 2 -> 1, 4 -> 2, 3 -> 3, 5 -> 4, 6 -> 5, 7 -> 6
  return code == 1 ? 0 : code == 2 ? 1 : code == 4 ? 2 : code == 3 ? 3 : code == 5 ? 4 : code == 6 ? 5 : 6;
}
__host__ __device__ constexpr int popc3(int c) { return (c & 1) + ((c >> 1) & 1) + ((c >> 2) & 1); }

// Corner c (0..3) of the six positively oriented tetrahedra:
//   (0,1,2): 0 1 3 7   (0,2,1): 0 5 1 7   (1,0,2): 0 3 2 7
//   (1,2,0): 0 2 6 7   (2,0,1): 0 4 5 7   (2,1,0): 0 6 4 7
__host__ __device__ constexpr int tet_corner(int tet, int c) {
  return c == 0 ? 0 : c == 3 ? 7 : (c == 1 ? (tet == 0 ? 1 : tet == 1 ? 5 : tet == 2 ? 3 : tet == 3 ? 2 : tet == 4 ? 4 : 6)
                                           : (tet == 0 ? 3 : tet == 1 ? 1 : tet == 2 ? 2 : tet == 3 ? 6 : tet == 4 ? 5 : 4));
}

__device__ inline int code_offset(int code, int res) {
  return (code & 1) + ((code >> 1) & 1) * res + ((code >> 2) & 1) * res * res;
}

// Edges of a node that carry a vertex, from its corner byte.
__device__ inline unsigned int edge_flags(unsigned int mask) {
  const unsigned int in0 = mask & 1u;
  unsigned int f = 0u;
#pragma unroll
  for (int d = 0; d < 7; ++d) f |= ((((mask >> dir_code(d)) & 1u) ^ in0) << d);
  return f;
}

// Inside mask of tetrahedron `tet` (bit c for corner q_c).
__device__ inline int tet_mask(int tet, unsigned int mask) {
  int m = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) m |= (int)((mask >> tet_corner(tet, c)) & 1u) << c;
  return m;
}
__device__ inline int tris_of_mask(int m) {
  const int n = __popc(m);
  return n == 2 ? 2 : (n == 1 || n == 3 ? 1 : 0);
}

// Triangles of the cube at a node (0 for nodes on the upper grid faces).
__device__ inline int cube_tri_count(bool full, unsigned int mask) {
  if (!full || mask == 0u || mask == 255u) return 0;
  int n = 0;
#pragma unroll
  for (int tet = 0; tet < 6; ++tet) n += tris_of_mask(tet_mask(tet, mask));
  return n;
}

// Per-workgroup tables over the 256 corner bytes: triangles of a full cube
// and vertices of a node.
struct MeshLut {
  uint8_t tris[256];
  uint8_t verts[256];
};

__device__ inline void build_lut(MeshLut& L) {
  for (int b = threadIdx.x; b < 256; b += blockDim.x) {
    L.tris[b] = (uint8_t)cube_tri_count(true, (unsigned int)b);
    L.verts[b] = (uint8_t)__popc(edge_flags((unsigned int)b));
  }
  __syncthreads();
}

constexpr int kScanThreads = 1024;

// Exclusive prefix of v over the workgroup; the workgroup total in `total`.
__device__ inline int block_exclusive(int v, int* lds, int& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  if (lane == 63) lds[w] = incl;
  __syncthreads();
  int pre = 0;
  total = 0;
  for (int i = 0; i < (int)(blockDim.x / 64); ++i) {
    const int s = lds[i];
    if (i < w) pre += s;
    total += s;
  }
  __syncthreads();
  return pre + incl - v;
}

// Inside bits of row (r, k) and (r, k + 1) at x and x + 1 for every lane of a
// wave: bit 0 (x, r, k), bit 1 (x + 1, r, k), bit 2 (x, r, k + 1), bit 3 (x + 1, r, k + 1).
__device__ inline unsigned int row_bits(const MeshArgs& A, int x, int r, int k, int lane) {
  const int res = A.res;
  const bool xin = x < res, x1 = x + 1 < res, k1 = k + 1 < res;
  const long long base0 = ((long long)k * res + r) * res, base1 = base0 + (long long)res * res;
  const bool a = xin && A.values[base0 + x] < A.iso;
  const bool b = xin && k1 && A.values[base1 + x] < A.iso;
  // lane 63 reads its x + 1 neighbour itself; the others take it from the ballot
  bool a1 = false, b1 = false;
  if (lane == 63 && x1) {
    a1 = A.values[base0 + x + 1] < A.iso;
    b1 = k1 && A.values[base1 + x + 1] < A.iso;
  }
  const unsigned long long ba = __ballot(a), bb = __ballot(b);
  if (lane < 63) {
    a1 = (ba >> (lane + 1)) & 1ull;
    b1 = (bb >> (lane + 1)) & 1ull;
  }
  return (a ? 1u : 0u) | (a1 ? 2u : 0u) | (b ? 4u : 0u) | (b1 ? 8u : 0u);
}

__global__ void __launch_bounds__(kMeshThreads) k_mt_mask(MeshArgs A) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int res = A.res;
  const int x = blockIdx.x * 64 + lane, k = blockIdx.z;
  const int j0 = (blockIdx.y * (kMeshThreads / 64) + w) * kMaskRows;
  if (j0 >= res) return;  // uniform per wave; no barriers follow
  const bool xin = x < res, x1 = x + 1 < res, k1 = k + 1 < res;
  // all kMaskRows + 1 rows first: their loads are in flight together
  unsigned int rb[kMaskRows + 1];
#pragma unroll
  for (int rr = 0; rr <= kMaskRows; ++rr) rb[rr] = j0 + rr < res ? row_bits(A, x, j0 + rr, k, lane) : 0u;
#pragma unroll
  for (int rr = 0; rr < kMaskRows; ++rr) {
    const int r = j0 + rr;
    if (r < res && xin) {
      const bool r1 = r + 1 < res;
      const unsigned int prev = rb[rr], next = rb[rr + 1];
      const unsigned int c0 = prev & 1u;
      // corner c: (dx, dy, dz) = (c & 1, c >> 1 & 1, c >> 2); dy selects the next row
      unsigned int m = c0;
      m |= (x1 ? (prev >> 1) & 1u : c0) << 1;
      m |= (r1 ? next & 1u : c0) << 2;
      m |= (x1 && r1 ? (next >> 1) & 1u : c0) << 3;
      m |= (k1 ? (prev >> 2) & 1u : c0) << 4;
      m |= (x1 && k1 ? (prev >> 3) & 1u : c0) << 5;
      m |= (r1 && k1 ? (next >> 2) & 1u : c0) << 6;
      m |= (x1 && r1 && k1 ? (next >> 3) & 1u : c0) << 7;
      A.mask[((long long)k * res + r) * res + x] = (uint8_t)m;
    }
  }
}

// The flat run of a thread: kFlat nodes from node0 (fewer at the end), with
// the grid position of node0.
struct Flat {
  int node0, len, i, j, k;
};

__device__ inline Flat flat_run(const MeshArgs& A) {
  Flat f{0, 0, 0, 0, 0};
  const long long node0 = ((long long)blockIdx.x * kMeshThreads + threadIdx.x) * kFlat;
  if (node0 < A.n_nodes) {
    f.node0 = (int)node0;
    f.len = min(kFlat, A.n_nodes - f.node0);
    const int row = f.node0 / A.res;
    f.i = f.node0 - row * A.res;
    f.j = row % A.res;
    f.k = row / A.res;
  }
  return f;
}

__device__ inline void flat_step(int res, int& i, int& j, int& k) {
  if (++i == res) {
    i = 0;
    if (++j == res) {
      j = 0;
      ++k;
    }
  }
}

// The corner bytes of a run (one 16-byte load when the run is whole).
__device__ inline void flat_masks(const MeshArgs& A, const Flat& f, unsigned int (&m)[kFlat / 4]) {
  if (f.len == kFlat) {
    const uint4 q = *(const uint4*)(A.mask + f.node0);
    m[0] = q.x;
    m[1] = q.y;
    m[2] = q.z;
    m[3] = q.w;
  } else {
#pragma unroll
    for (int w = 0; w < kFlat / 4; ++w) m[w] = 0u;
    for (int x = 0; x < f.len; ++x) m[x >> 2] |= (unsigned int)A.mask[f.node0 + x] << (8 * (x & 3));
  }
}

__device__ inline unsigned int byte_of(const unsigned int (&m)[kFlat / 4], int x) {
  return (m[x >> 2] >> (8 * (x & 3))) & 255u;
}

// Vertices and triangles of a thread's run (nodes on the upper grid faces
// hold no cube); also the number of nodes with triangles.
__device__ inline void run_counts(const MeshArgs& A, const MeshLut& L, const Flat& f,
                                  const unsigned int (&m)[kFlat / 4], int& nv, int& nt, int& ns) {
  nv = nt = ns = 0;
  if (f.len <= 0) return;
  const int res = A.res;
  int i = f.i, j = f.j, k = f.k;
#pragma unroll
  for (int x = 0; x < kFlat; ++x) {
    const unsigned int b = byte_of(m, x);  // 0 past the end of a short run
    nv += L.verts[b];
    const int c = (i + 1 < res && j + 1 < res && k + 1 < res) ? L.tris[b] : 0;
    nt += c;
    ns += c ? 1 : 0;
    flat_step(res, i, j, k);
  }
}

__global__ void __launch_bounds__(kMeshThreads) k_mt_count(MeshArgs A) {
  __shared__ int lds[2][kMeshThreads / 64];
  __shared__ MeshLut L;
  build_lut(L);
  const Flat f = flat_run(A);
  unsigned int m[kFlat / 4] = {0u, 0u, 0u, 0u};
  if (f.len > 0) flat_masks(A, f, m);
  int nv, nt, ns;
  run_counts(A, L, f, m, nv, nt, ns);
  if (!__syncthreads_or(nv | nt)) {
    if (threadIdx.x == 0) {
      A.bsum_v[blockIdx.x] = 0;
      A.bsum_t[blockIdx.x] = 0;
    }
    return;
  }
  int tv, tt;
  block_exclusive(nv, lds[0], tv);
  block_exclusive(nt, lds[1], tt);
  if (threadIdx.x == 0) {
    A.bsum_v[blockIdx.x] = tv;
    A.bsum_t[blockIdx.x] = tt;
  }
}

// Two-level exclusive scan of the per-workgroup counts: groups of
// kScanThreads block sums are scanned in place (group totals to gsum), then one
// workgroup scans the group totals and writes the grand totals to counts.  The
// offset of block b is then bsum[b] + gsum[b / kScanThreads].
__global__ void __launch_bounds__(kScanThreads) k_mt_scan_blocks(MeshArgs A) {
  __shared__ int lds[2][kScanThreads / 64];
  const int b = blockIdx.x * kScanThreads + threadIdx.x;
  const int xv = b < A.n_blocks ? A.bsum_v[b] : 0, xt = b < A.n_blocks ? A.bsum_t[b] : 0;
  int tv, tt;
  const int rv = block_exclusive(xv, lds[0], tv);
  const int rt = block_exclusive(xt, lds[1], tt);
  if (b < A.n_blocks) {
    A.bsum_v[b] = rv;
    A.bsum_t[b] = rt;
  }
  if (threadIdx.x == 0) {
    A.gsum_v[blockIdx.x] = tv;
    A.gsum_t[blockIdx.x] = tt;
  }
}

__global__ void __launch_bounds__(kScanThreads) k_mt_scan_groups(MeshArgs A) {
  __shared__ int lds[2][kScanThreads / 64];
  const int g = threadIdx.x;
  const int xv = g < A.n_groups ? A.gsum_v[g] : 0, xt = g < A.n_groups ? A.gsum_t[g] : 0;
  int tv, tt;
  const int rv = block_exclusive(xv, lds[0], tv);
  const int rt = block_exclusive(xt, lds[1], tt);
  if (g < A.n_groups) {
    A.gsum_v[g] = rv;
    A.gsum_t[g] = rt;
  }
  if (g == 0) {
    A.counts[0] = tv;
    A.counts[1] = tt;
  }
}

// Work list of a workgroup: its surface nodes in node order, each with the
// id of its first vertex (or triangle), filled from the per-thread prefixes.
constexpr int kListMax = kMeshThreads * kFlat;
struct MeshList {
  int node[kListMax];
  int first[kListMax];
};

__global__ void __launch_bounds__(kMeshThreads) k_mt_verts(MeshArgs A) {
  __shared__ int lds[2][kMeshThreads / 64];
  __shared__ MeshLut L;
  __shared__ MeshList W;
  build_lut(L);
  const int res = A.res;
  const Flat f = flat_run(A);
  unsigned int m[kFlat / 4] = {0u, 0u, 0u, 0u};
  if (f.len > 0) flat_masks(A, f, m);
  int nv = 0, ns = 0;
#pragma unroll
  for (int x = 0; x < kFlat; ++x) {
    const int c = L.verts[byte_of(m, x)];
    nv += c;
    ns += c ? 1 : 0;
  }
  if (!__syncthreads_or(nv)) return;
  int total, n_list;
  int id = A.bsum_v[blockIdx.x] + A.gsum_v[blockIdx.x / kScanThreads] + block_exclusive(nv, lds[0], total);
  int pos = block_exclusive(ns, lds[1], n_list);
  for (int x = 0; x < f.len; ++x) {
    const int c = L.verts[byte_of(m, x)];
    if (c) {
      W.node[pos] = f.node0 + x;
      W.first[pos] = id;
      ++pos;
      id += c;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n_list; e += kMeshThreads) {
    const int node = W.node[e];
    int vid = W.first[e];
    const unsigned int flags = edge_flags(A.mask[node]);
    A.vert_off[node] = vid;  // read back only for nodes that carry vertices
    const int row = node / res;
    const int i = node - row * res, j = row % res, k = row / res;
    const float v0 = A.values[node];
    float v1[7];
#pragma unroll
    for (int d = 0; d < 7; ++d) v1[d] = ((flags >> d) & 1u) ? A.values[node + code_offset(dir_code(d), res)] : 0.f;
    const float x0 = grid_coord(A.lo, A.hi, res, i), y0 = grid_coord(A.lo, A.hi, res, j),
                z0 = grid_coord(A.lo, A.hi, res, k);
#pragma unroll
    for (int d = 0; d < 7; ++d) {
      if (!((flags >> d) & 1u)) continue;
      if (vid < A.max_v) {
        const int c = dir_code(d);
        const float t = (A.iso - v0) / (v1[d] - v0);
        const float x1 = grid_coord(A.lo, A.hi, res, i + (c & 1));
        const float y1 = grid_coord(A.lo, A.hi, res, j + ((c >> 1) & 1));
        const float z1 = grid_coord(A.lo, A.hi, res, k + ((c >> 2) & 1));
        A.verts[3LL * vid + 0] = fmaf(t, x1 - x0, x0);
        A.verts[3LL * vid + 1] = fmaf(t, y1 - y0, y0);
        A.verts[3LL * vid + 2] = fmaf(t, z1 - z0, z0);
      }
      ++vid;
    }
  }
}

__device__ inline void put_tri(const MeshArgs& A, int t, int a, int b, int c) {
  if (t < A.max_t) {
    A.tris[3LL * t + 0] = a;
    A.tris[3LL * t + 1] = b;
    A.tris[3LL * t + 2] = c;
  }
}

// Index of the corner pair {p, q} (p != q) among (0,1) (0,2) (0,3) (1,2) (1,3) (2,3).
__device__ inline int pair_index(int p, int q) {
  const int lo = min(p, q), hi = max(p, q);
  return lo == 0 ? hi - 1 : (lo == 1 ? hi + 1 : 5);
}
__device__ inline int pick6(int i, const int (&e)[6]) {
  return i == 0 ? e[0] : i == 1 ? e[1] : i == 2 ? e[2] : i == 3 ? e[3] : i == 4 ? e[4] : e[5];
}

// Triangles of the cube at `node` with corner byte `mask`; gv / gf are the
// first vertex ids and edge flags of the cube's corners 0..6.
__device__ inline void emit_cube(const MeshArgs& A, unsigned int mask, const int (&gv)[7], const unsigned int (&gf)[7],
                                 int& t) {
#pragma unroll
  for (int tet = 0; tet < 6; ++tet) {
    const int m = tet_mask(tet, mask);
    const int n_in = __popc(m);
    if (n_in == 0 || n_in == 4) continue;
    // vertex ids of the tetrahedron's six edges (constant corner codes)
    int e[6];
#pragma unroll
    for (int pi = 0; pi < 6; ++pi) {
      const int p = pi < 3 ? 0 : (pi < 5 ? 1 : 2), q = pi < 3 ? pi + 1 : (pi < 5 ? pi - 1 : 3);
      const int u = tet_corner(tet, p), w = tet_corner(tet, q);
      const int lower = popc3(u) < popc3(w) ? u : w;
      const int d = code_dir(u ^ w);
      e[pi] = gv[lower] + __popc(gf[lower] & ((1u << d) - 1u));
    }
    if (n_in == 1 || n_in == 3) {
      // the corner alone on its side, then the others in increasing order,
      // the last two swapped for odd a: (a b c d) is an even permutation
      const int a = __ffs(n_in == 1 ? m : (~m & 15)) - 1;
      const int r0 = a == 0 ? 1 : 0;
      int r1 = a <= 1 ? 2 : 1, r2 = a <= 2 ? 3 : 2;
      if (a & 1) {
        const int tmp = r1;
        r1 = r2;
        r2 = tmp;
      }
      const int eb = pick6(pair_index(a, r0), e), ec = pick6(pair_index(a, r1), e), ed = pick6(pair_index(a, r2), e);
      if (n_in == 1)
        put_tri(A, t, eb, ec, ed);
      else
        put_tri(A, t, eb, ed, ec);
      ++t;
    } else {
      const int a = __ffs(m) - 1, b = 31 - __clz(m);  // inside corners, a < b
      const int om = ~m & 15;
      int c = __ffs(om) - 1, d = 31 - __clz(om);  // outside corners, c < d
      if ((a == 0 && b == 2) || (a == 1 && b == 3)) {
        const int tmp = c;
        c = d;
        d = tmp;
      }
      const int e_ac = pick6(pair_index(a, c), e), e_ad = pick6(pair_index(a, d), e);
      const int e_bd = pick6(pair_index(b, d), e), e_bc = pick6(pair_index(b, c), e);
      put_tri(A, t, e_ac, e_ad, e_bd);
      put_tri(A, t + 1, e_ac, e_bd, e_bc);
      t += 2;
    }
  }
}

__global__ void __launch_bounds__(kMeshThreads) k_mt_tris(MeshArgs A) {
  __shared__ int lds[2][kMeshThreads / 64];
  __shared__ MeshLut L;
  __shared__ MeshList W;
  build_lut(L);
  const int res = A.res;
  const Flat f = flat_run(A);
  unsigned int m[kFlat / 4] = {0u, 0u, 0u, 0u};
  if (f.len > 0) flat_masks(A, f, m);
  int nv, nt, ns;
  run_counts(A, L, f, m, nv, nt, ns);
  if (!__syncthreads_or(nt)) return;
  int total, n_list;
  int t = A.bsum_t[blockIdx.x] + A.gsum_t[blockIdx.x / kScanThreads] + block_exclusive(nt, lds[0], total);
  int pos = block_exclusive(ns, lds[1], n_list);
  if (nt) {
    int i = f.i, j = f.j, k = f.k;
    for (int x = 0; x < f.len; ++x) {
      const int c = (i + 1 < res && j + 1 < res && k + 1 < res) ? L.tris[byte_of(m, x)] : 0;
      if (c) {
        W.node[pos] = f.node0 + x;
        W.first[pos] = t;
        ++pos;
        t += c;
      }
      flat_step(res, i, j, k);
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n_list; e += kMeshThreads) {
    const int node = W.node[e];
    int tt = W.first[e];
    const unsigned int mask = A.mask[node];
    // first vertex ids and edge flags of the corners 0..6, in one round trip
    int gv[7];
    unsigned int gf[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) {
      const int q = node + code_offset(c, res);
      gv[c] = A.vert_off[q];
      gf[c] = edge_flags(A.mask[q]);
    }
    emit_cube(A, mask, gv, gf, tt);
  }
}

// Workgroups of the flat passes for a grid side.
int mesh_blocks(int res) {
  const long long nodes = (long long)res * res * res;
  return (int)((nodes + (long long)kMeshThreads * kFlat - 1) / ((long long)kMeshThreads * kFlat));
}

hipError_t launch_marching_tets(const MeshArgs& a, hipStream_t s) {
  const int rows_per_block = (kMeshThreads / 64) * kMaskRows;
  const dim3 mgrid((a.res + 63) / 64, (a.res + rows_per_block - 1) / rows_per_block, a.res);
  hipLaunchKernelGGL(k_mt_mask, mgrid, dim3(kMeshThreads), 0, s, a);
  const dim3 grid(a.n_blocks), block(kMeshThreads);
  hipLaunchKernelGGL(k_mt_count, grid, block, 0, s, a);
  hipLaunchKernelGGL(k_mt_scan_blocks, dim3(a.n_groups), dim3(kScanThreads), 0, s, a);
  hipLaunchKernelGGL(k_mt_scan_groups, dim3(1), dim3(kScanThreads), 0, s, a);
  hipLaunchKernelGGL(k_mt_verts, grid, block, 0, s, a);
  hipLaunchKernelGGL(k_mt_tris, grid, block, 0, s, a);
  return hipGetLastError();
}

}  // namespace nnm

/*
 * mesh_oracle.c -- plain CPU extraction of a triangle mesh from a grid of
 * scene-function values, the coarse surface that neural normal mapping (Sec. 5)
 * decorates with the normals of a finer network (the triangle-mesh example of
 * Sec. 5 and Fig. 5, where the coarse mesh is extracted from a (64,1) network).
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load or call this code; the GPU library never does,
 * and the two share no code.
 *
 * The paper extracts its coarse mesh with marching cubes and does not fix the
 * variant.  This build uses marching tetrahedra on the Kuhn (Freudenthal)
 * subdivision of every grid cube, which gives a closed, consistently oriented
 * piecewise-linear surface without case tables.  The output is fully specified
 * so that any implementation produces the same arrays:
 *
 *   grid      node (i, j, k), 0 <= i, j, k < res, linear index (k res + j) res + i;
 *             coordinate of index i: lo + (hi - lo) i / (res - 1).
 *   inside    value < iso (a NaN value is outside).
 *   edges     seven per node, from the node to node + D, D in the order
 *             (1,0,0) (0,1,0) (0,0,1) (1,1,0) (1,0,1) (0,1,1) (1,1,1); an edge
 *             whose ends differ in inside-ness carries one vertex at the zero of
 *             the linear interpolant, x0 + (iso - v0) / (v1 - v0) (x1 - x0).
 *             Vertices are numbered in (node index, edge order).
 *   tets      cube with lower corner (i, j, k) (all < res - 1), six tetrahedra,
 *             one per axis order (a, b, c) in lexicographic order: corners
 *             0, e_a, e_a + e_b, (1,1,1); for odd orders the middle two corners
 *             are swapped so that every tetrahedron is positively oriented.
 *             Cubes are visited in node order, tetrahedra in the order above.
 *   triangles per tetrahedron (q0 q1 q2 q3), with E(u, w) the vertex of edge uw:
 *             one corner a alone on its side: (b, c, d) the other corners in
 *             increasing order, c and d swapped when a is odd, so that (a b c d)
 *             is an even permutation; one inside corner gives
 *             (E(a,b), E(a,c), E(a,d)), one outside corner (E(a,b), E(a,d), E(a,c));
 *             two inside corners a < b, outside c < d, c and d swapped when
 *             {a, b} is {0, 2} or {1, 3}: (E(a,c), E(a,d), E(b,d)) and
 *             (E(a,c), E(b,d), E(b,c)).
 *             Every triangle then faces from the inside to the outside.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static const int kDir[7][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1}};
static const int kOrder[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
static const int kOrderOdd[6] = {0, 1, 1, 0, 0, 1};

static double coord(double lo, double hi, int res, int i) { return lo + (hi - lo) * (double)i / (double)(res - 1); }

static int inside_at(const float* v, float iso, int64_t node) { return v[node] < iso; }

/* Index of the edge direction with components (dx, dy, dz), each 0 or 1. */
static int dir_index(int dx, int dy, int dz) {
  for (int d = 0; d < 7; ++d)
    if (kDir[d][0] == dx && kDir[d][1] == dy && kDir[d][2] == dz) return d;
  return -1;
}

/* Vertex id of the edge between two corners of the cube at (i, j, k); corners
   are given as offsets in {0,1}^3, one componentwise below the other. */
static int64_t edge_vertex(const int32_t* edge_id, int res, int i, int j, int k, const int u[3], const int w[3]) {
  const int* lower = (u[0] + u[1] + u[2] <= w[0] + w[1] + w[2]) ? u : w;
  const int* upper = lower == u ? w : u;
  const int d = dir_index(upper[0] - lower[0], upper[1] - lower[1], upper[2] - lower[2]);
  const int64_t node = ((int64_t)(k + lower[2]) * res + (j + lower[1])) * res + (i + lower[0]);
  return edge_id[node * 7 + d];
}

/* counts[0] = vertices, counts[1] = triangles (the full totals); the first
   cap_v vertices and cap_t triangles are written when the arrays are given.
   Returns 0, or -1 on bad arguments, a grid whose 7 res^3 edge ids overflow
   int32, or allocation failure. */
int orc_marching_tets(const float* values, int res, double lo, double hi, float iso, double* verts, int32_t* tris,
                      int64_t cap_v, int64_t cap_t, int64_t* counts) {
  if (!values || !counts || res < 2) return -1;
  const int64_t n_nodes = (int64_t)res * res * res;
  if (n_nodes * 7 > INT32_MAX) return -1; /* vertex ids are int32 */
  int32_t* edge_id = (int32_t*)malloc((size_t)n_nodes * 7 * sizeof(int32_t));
  if (!edge_id) return -1;

  /* vertices, numbered in (node, edge) order */
  int64_t nv = 0;
  for (int k = 0; k < res; ++k)
    for (int j = 0; j < res; ++j)
      for (int i = 0; i < res; ++i) {
        const int64_t node = ((int64_t)k * res + j) * res + i;
        for (int d = 0; d < 7; ++d) {
          edge_id[node * 7 + d] = -1;
          const int i1 = i + kDir[d][0], j1 = j + kDir[d][1], k1 = k + kDir[d][2];
          if (i1 >= res || j1 >= res || k1 >= res) continue;
          const int64_t other = ((int64_t)k1 * res + j1) * res + i1;
          if (inside_at(values, iso, node) == inside_at(values, iso, other)) continue;
          if (verts && nv < cap_v) {
            const double v0 = values[node], v1 = values[other];
            const double t = ((double)iso - v0) / (v1 - v0);
            const double p0[3] = {coord(lo, hi, res, i), coord(lo, hi, res, j), coord(lo, hi, res, k)};
            const double p1[3] = {coord(lo, hi, res, i1), coord(lo, hi, res, j1), coord(lo, hi, res, k1)};
            for (int c = 0; c < 3; ++c) verts[3 * nv + c] = p0[c] + t * (p1[c] - p0[c]);
          }
          edge_id[node * 7 + d] = (int32_t)nv++;
        }
      }

  /* triangles, cube by cube, tetrahedron by tetrahedron */
  int64_t nt = 0;
  for (int k = 0; k + 1 < res; ++k)
    for (int j = 0; j + 1 < res; ++j)
      for (int i = 0; i + 1 < res; ++i)
        for (int tet = 0; tet < 6; ++tet) {
          int q[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {1, 1, 1}};
          const int a = kOrder[tet][0], b = kOrder[tet][1];
          q[1][a] = 1;
          q[2][a] = 1;
          q[2][b] = 1;
          if (kOrderOdd[tet]) {
            for (int c = 0; c < 3; ++c) {
              const int tmp = q[1][c];
              q[1][c] = q[2][c];
              q[2][c] = tmp;
            }
          }
          int in[4], n_in = 0;
          for (int c = 0; c < 4; ++c) {
            const int64_t node = ((int64_t)(k + q[c][2]) * res + (j + q[c][1])) * res + (i + q[c][0]);
            in[c] = inside_at(values, iso, node);
            n_in += in[c];
          }
          int64_t tri[2][3];
          int ntri = 0;
          if (n_in == 1 || n_in == 3) {
            const int lone = n_in == 1 ? 1 : 0; /* the side that has one corner */
            int ca = -1;
            for (int c = 0; c < 4; ++c)
              if (in[c] == lone) ca = c;
            int rest[3], r = 0;
            for (int c = 0; c < 4; ++c)
              if (c != ca) rest[r++] = c;
            if (ca & 1) {
              const int tmp = rest[1];
              rest[1] = rest[2];
              rest[2] = tmp;
            }
            const int64_t eb = edge_vertex(edge_id, res, i, j, k, q[ca], q[rest[0]]);
            const int64_t ec = edge_vertex(edge_id, res, i, j, k, q[ca], q[rest[1]]);
            const int64_t ed = edge_vertex(edge_id, res, i, j, k, q[ca], q[rest[2]]);
            tri[0][0] = eb;
            tri[0][1] = n_in == 1 ? ec : ed;
            tri[0][2] = n_in == 1 ? ed : ec;
            ntri = 1;
          } else if (n_in == 2) {
            int ins[2], outs[2], ni = 0, no = 0;
            for (int c = 0; c < 4; ++c) {
              if (in[c])
                ins[ni++] = c;
              else
                outs[no++] = c;
            }
            const int ca = ins[0], cb = ins[1];
            int cc = outs[0], cd = outs[1];
            if ((ca == 0 && cb == 2) || (ca == 1 && cb == 3)) {
              const int tmp = cc;
              cc = cd;
              cd = tmp;
            }
            const int64_t e_ac = edge_vertex(edge_id, res, i, j, k, q[ca], q[cc]);
            const int64_t e_ad = edge_vertex(edge_id, res, i, j, k, q[ca], q[cd]);
            const int64_t e_bd = edge_vertex(edge_id, res, i, j, k, q[cb], q[cd]);
            const int64_t e_bc = edge_vertex(edge_id, res, i, j, k, q[cb], q[cc]);
            tri[0][0] = e_ac;
            tri[0][1] = e_ad;
            tri[0][2] = e_bd;
            tri[1][0] = e_ac;
            tri[1][1] = e_bd;
            tri[1][2] = e_bc;
            ntri = 2;
          }
          for (int t = 0; t < ntri; ++t) {
            if (tris && nt < cap_t)
              for (int c = 0; c < 3; ++c) tris[3 * nt + c] = (int32_t)tri[t][c];
            ++nt;
          }
        }
  free(edge_id);
  counts[0] = nv;
  counts[1] = nt;
  return 0;
}

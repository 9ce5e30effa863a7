// Mesh hand-off: Marching Cubes over the surface cells of a labelled grid (the mesh
// extraction of the PIFu baseline the paper accelerates, Sec. 1 and Sec. 3.2 "Inference
// for Human Reconstruction"), with vertex colours: the input pixel where the vertex is
// visible from the input camera, Eq. 2's colour network elsewhere (the texture paragraph
// of Sec. 3.1).
//
// Conventions:
//   * corner c of a cell has offsets (c >> 2 & 1, c >> 1 & 1, c & 1) along (x, y, z);
//     local edge e = 4 * axis + 2 * u + v, (u, v) the offsets of its lower corner along
//     the other two axes in increasing axis order;
//   * each face is cut by segments between its crossing edges; a face whose corners
//     alternate (ambiguous) keeps its inside corners apart; a segment is directed so
//     that, seen from outside the cube, the face's inside corners lie on its left;
//   * segments join into loops; each loop, listed from its smallest edge, is cut into the
//     fan (v0, v[i+1], v[i]) from the first position v0 whose fan has no triangle lying in
//     one cube face: normals point from label 1 to label 0;
//   * one vertex per lattice edge whose end labels differ, at the 0.5 crossing of the
//     linear interpolation of the end occupancies; vertices sorted by edge id 3 n + axis.
#include "pifu_internal.h"

namespace pifu {

// Triangle table: for each corner case, the number of triangles and their local edges.
__constant__ uint8_t c_mc_ntri[256];
__constant__ uint8_t c_mc_edge[256][15];

namespace {

inline unsigned grid1d(size_t n, int block) { return (unsigned)((n + block - 1) / block); }

// ---------------------------------------------------------------- table (host)
// Doubled integer coordinates: corner c -> 2 * offsets, edge midpoint -> lo + hi.
struct V3 {
  int x, y, z;
};
V3 corner2(int c) { return V3{2 * ((c >> 2) & 1), 2 * ((c >> 1) & 1), 2 * (c & 1)}; }
int axis_bit(int axis) { return 2 - axis; }   // bit of corner c holding the axis offset
void edge_ends(int e, int& lo, int& hi) {
  const int axis = e >> 2, u = (e >> 1) & 1, v = e & 1;
  int off[3] = {0, 0, 0};
  int q = 0;
  for (int a = 0; a < 3; ++a)
    if (a != axis) off[a] = q++ == 0 ? u : v;
  lo = (off[0] << 2) | (off[1] << 1) | off[2];
  off[axis] = 1;
  hi = (off[0] << 2) | (off[1] << 1) | off[2];
}
V3 edge_mid2(int e) {
  int a, b;
  edge_ends(e, a, b);
  const V3 p = corner2(a), q = corner2(b);
  return V3{(p.x + q.x) / 2, (p.y + q.y) / 2, (p.z + q.z) / 2};
}
// faces of the cube containing both ends of edge e: bit 2 * axis + side
int edge_faces(int e) {
  int a, b, m = 0;
  edge_ends(e, a, b);
  for (int ax = 0; ax < 3; ++ax)
    for (int sd = 0; sd < 2; ++sd)
      if (((a >> axis_bit(ax)) & 1) == sd && ((b >> axis_bit(ax)) & 1) == sd) m |= 1 << (2 * ax + sd);
  return m;
}

int build_case(int cs, uint8_t* out) {
  int succ[12];
  for (int e = 0; e < 12; ++e) succ[e] = -1;
  for (int ax = 0; ax < 3; ++ax) {
    for (int sd = 0; sd < 2; ++sd) {
      int nrm[3] = {0, 0, 0};
      nrm[ax] = sd ? 1 : -1;
      int cross_e[4], nc = 0, ins[4], ni = 0;
      for (int e = 0; e < 12; ++e) {
        if ((e >> 2) == ax) continue;
        int a, b;
        edge_ends(e, a, b);
        if (((a >> axis_bit(ax)) & 1) != sd) continue;   // both ends share the face coordinate
        if (((cs >> a) & 1) != ((cs >> b) & 1)) cross_e[nc++] = e;
      }
      for (int c = 0; c < 8; ++c)
        if (((c >> axis_bit(ax)) & 1) == sd && ((cs >> c) & 1)) ins[ni++] = c;
      int sa[2], sb[2], sq[2], ns = 0;
      if (nc == 2) {
        sa[0] = cross_e[0];
        sb[0] = cross_e[1];
        sq[0] = ins[0];
        ns = 1;
      } else if (nc == 4) {
        for (int i = 0; i < ni; ++i) {   // one segment around each inside corner
          int got = 0, pair[2];
          for (int k = 0; k < 4; ++k) {
            int a, b;
            edge_ends(cross_e[k], a, b);
            if (a == ins[i] || b == ins[i]) pair[got++] = cross_e[k];
          }
          sa[ns] = pair[0];
          sb[ns] = pair[1];
          sq[ns] = ins[i];
          ++ns;
        }
      }
      for (int k = 0; k < ns; ++k) {
        const V3 A = edge_mid2(sa[k]), B = edge_mid2(sb[k]), Q = corner2(sq[k]);
        const int d[3] = {B.x - A.x, B.y - A.y, B.z - A.z};
        const int w[3] = {Q.x - A.x, Q.y - A.y, Q.z - A.z};
        const int cr[3] = {nrm[1] * d[2] - nrm[2] * d[1], nrm[2] * d[0] - nrm[0] * d[2],
                           nrm[0] * d[1] - nrm[1] * d[0]};
        const int side = cr[0] * w[0] + cr[1] * w[1] + cr[2] * w[2];
        if (side > 0) succ[sa[k]] = sb[k];
        else succ[sb[k]] = sa[k];
      }
    }
  }
  int nt = 0;
  bool seen[12] = {};
  for (int st = 0; st < 12; ++st) {
    if (succ[st] < 0 || seen[st]) continue;
    int loop[12], len = 0;
    int e = st;
    do {
      loop[len++] = e;
      seen[e] = true;
      e = succ[e];
    } while (e != st && len < 12);
    int origin = -1;
    for (int o = 0; o < len && origin < 0; ++o) {
      bool flat = false;
      for (int i = 1; i + 1 < len; ++i) {
        const int a = loop[o], b = loop[(o + i + 1) % len], c = loop[(o + i) % len];
        if (edge_faces(a) & edge_faces(b) & edge_faces(c)) flat = true;
      }
      if (!flat) origin = o;
    }
    if (origin < 0) return -1;
    for (int i = 1; i + 1 < len; ++i) {
      out[3 * nt + 0] = (uint8_t)loop[origin];
      out[3 * nt + 1] = (uint8_t)loop[(origin + i + 1) % len];
      out[3 * nt + 2] = (uint8_t)loop[(origin + i) % len];
      ++nt;
    }
  }
  return nt;
}

// ---------------------------------------------------------------- kernels
__device__ inline void node_ijk(uint32_t n, int nn, int& i, int& j, int& k) {
  const uint32_t nyz = (uint32_t)nn * nn;
  i = (int)(n / nyz);
  const uint32_t r = n - (uint32_t)i * nyz;
  j = (int)(r / nn);
  k = (int)(r - (uint32_t)j * nn);
}

// flags[3 n + axis] = the lattice edge from node n along axis joins different labels.
__global__ void __launch_bounds__(256)
k_mesh_edge_flags(const uint8_t* __restrict__ labels, int nn, uint8_t* __restrict__ flags) {
  const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t total = (uint32_t)nn * nn * nn;
  if (n >= total) return;
  int i, j, k;
  node_ijk(n, nn, i, j, k);
  const uint8_t l = labels[n];
  const uint32_t nyz = (uint32_t)nn * nn;
  flags[3 * (size_t)n + 0] = (i + 1 < nn) && labels[n + nyz] != l;
  flags[3 * (size_t)n + 1] = (j + 1 < nn) && labels[n + nn] != l;
  flags[3 * (size_t)n + 2] = (k + 1 < nn) && labels[n + 1] != l;
}

// kf[i nn + j] = largest k with label 1 in column (i, j), -1 if none.
__global__ void __launch_bounds__(256)
k_mesh_front(const uint8_t* __restrict__ labels, int nn, int32_t* __restrict__ kf) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (uint32_t)nn * nn) return;
  const uint8_t* col = labels + (size_t)c * nn;
  int k = nn - 1;
  while (k >= 0 && !col[k]) --k;
  kf[c] = k;
}

// Vertex m on edge ids[m]: its position, whether the input camera (orthographic, at
// z = +1) sees it (every column of the edge's nodes has its front node at or below the
// edge's k), and the point (x, y, z, 0.5) the colour network reads.
__global__ void __launch_bounds__(256)
k_mesh_verts(const uint32_t* __restrict__ ids, uint32_t nv, const float* __restrict__ occ,
             int nn, const int32_t* __restrict__ kf, float* __restrict__ verts,
             uint8_t* __restrict__ hidden, float4* __restrict__ pts) {
  const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nv) return;
  const uint32_t g = ids[m];
  const int axis = (int)(g % 3);
  const uint32_t na = g / 3;
  int i, j, k;
  node_ijk(na, nn, i, j, k);
  const uint32_t step = axis == 0 ? (uint32_t)nn * nn : (axis == 1 ? (uint32_t)nn : 1u);
  const double pa = occ[na], pb = occ[na + step];
  double t = pb == pa ? 0.5 : (0.5 - pa) / (pb - pa);
  t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
  const double h = 2.0 / (double)(nn - 1);
  double P[3] = {-1.0 + h * i, -1.0 + h * j, -1.0 + h * k};
  P[axis] += t * h;
  verts[3 * (size_t)m + 0] = (float)P[0];
  verts[3 * (size_t)m + 1] = (float)P[1];
  verts[3 * (size_t)m + 2] = (float)P[2];
  bool vis = kf[(size_t)i * nn + j] <= k;
  if (axis == 0) vis = vis && kf[(size_t)(i + 1) * nn + j] <= k;
  if (axis == 1) vis = vis && kf[(size_t)i * nn + j + 1] <= k;
  if (hidden) hidden[m] = !vis;
  if (pts) pts[m] = make_float4((float)P[0], (float)P[1], (float)P[2], 0.5f);
}

// Corner case of cell (i, j, k) from the labels.
__device__ inline int cell_case(const uint8_t* __restrict__ labels, int nn, int i, int j, int k) {
  int cs = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int x = i + ((c >> 2) & 1), y = j + ((c >> 1) & 1), z = k + (c & 1);
    if (labels[((size_t)x * nn + y) * nn + z]) cs |= 1 << c;
  }
  return cs;
}

__device__ inline void cell_ijk(uint32_t cell, int R, int& i, int& j, int& k) {
  const uint32_t rr = (uint32_t)R * R;
  i = (int)(cell / rr);
  const uint32_t r = cell - (uint32_t)i * rr;
  j = (int)(r / R);
  k = (int)(r - (uint32_t)j * R);
}

__global__ void __launch_bounds__(256)
k_mesh_tri_count(const uint32_t* __restrict__ cells, uint32_t nc, const uint8_t* __restrict__ labels,
                 int nn, uint32_t* __restrict__ cnt) {
  const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nc) return;
  int i, j, k;
  cell_ijk(cells[m], nn - 1, i, j, k);
  cnt[m] = c_mc_ntri[cell_case(labels, nn, i, j, k)];
}

// Triangles of cell m at off[m]: each local edge -> global edge id -> vertex index (binary
// search in the sorted edge ids).
__global__ void __launch_bounds__(256)
k_mesh_tri_write(const uint32_t* __restrict__ cells, uint32_t nc, const uint8_t* __restrict__ labels,
                 int nn, const uint32_t* __restrict__ off, const uint32_t* __restrict__ ids,
                 uint32_t nv, uint32_t* __restrict__ tris, uint32_t tri_cap) {
  const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nc) return;
  int i, j, k;
  cell_ijk(cells[m], nn - 1, i, j, k);
  const int cs = cell_case(labels, nn, i, j, k);
  const int nt = c_mc_ntri[cs];
  for (int t = 0; t < nt; ++t) {
    const uint32_t slot = off[m] + t;
    if (slot >= tri_cap) return;
    for (int q = 0; q < 3; ++q) {
      const int e = c_mc_edge[cs][3 * t + q];
      const int axis = e >> 2, u = (e >> 1) & 1, v = e & 1;
      int o[3] = {0, 0, 0};
      if (axis == 0) { o[1] = u; o[2] = v; }
      else if (axis == 1) { o[0] = u; o[2] = v; }
      else { o[0] = u; o[1] = v; }
      const uint32_t node = ((uint32_t)(i + o[0]) * nn + (uint32_t)(j + o[1])) * nn + (uint32_t)(k + o[2]);
      const uint32_t g = 3 * node + axis;
      uint32_t lo = 0, hi = nv;
      while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (ids[mid] < g) lo = mid + 1;
        else hi = mid;
      }
      tris[3 * (size_t)slot + q] = lo;
    }
  }
}

// Visible vertices take the input pixel: bilinear blend of the HWC image (3 channels),
// pixel u = (x+1)/2 (W-1), v = (y+1)/2 (H-1), texels outside the image 0.
__global__ void __launch_bounds__(256)
k_mesh_pixel_colors(const float* __restrict__ verts, const uint8_t* __restrict__ hidden, uint32_t nv,
                    const float* __restrict__ img, int H, int W, float* __restrict__ colors) {
  const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nv || hidden[m]) return;
  const double u = ((double)verts[3 * (size_t)m] + 1.0) * 0.5 * (W - 1);
  const double v = ((double)verts[3 * (size_t)m + 1] + 1.0) * 0.5 * (H - 1);
  const double fu0 = floor(u), fv0 = floor(v);
  const double fu = u - fu0, fv = v - fv0;
  const int u0 = (int)fu0, v0 = (int)fv0;
  const double w[4] = {(1.0 - fu) * (1.0 - fv), fu * (1.0 - fv), (1.0 - fu) * fv, fu * fv};
  const int tu[4] = {u0, u0 + 1, u0, u0 + 1};
  const int tv[4] = {v0, v0, v0 + 1, v0 + 1};
  double acc[3] = {0.0, 0.0, 0.0};
  for (int t = 0; t < 4; ++t) {
    if (tu[t] < 0 || tu[t] > W - 1 || tv[t] < 0 || tv[t] > H - 1) continue;
    const float* p = img + ((size_t)tv[t] * W + tu[t]) * 3;
    for (int c = 0; c < 3; ++c) acc[c] += w[t] * (double)p[c];
  }
  for (int c = 0; c < 3; ++c) colors[3 * (size_t)m + c] = (float)acc[c];
}

}  // namespace

int mesh_table_upload() {
  static uint8_t ntri[256];
  static uint8_t edge[256][15];
  for (int cs = 0; cs < 256; ++cs) {
    uint8_t out[36] = {};
    const int nt = build_case(cs, out);
    if (nt < 0 || nt > 5) return PIFU_ERR_UNSUPPORTED;
    ntri[cs] = (uint8_t)nt;
    for (int q = 0; q < 15; ++q) edge[cs][q] = q < 3 * nt ? out[q] : 0;
  }
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_mc_ntri), ntri, sizeof(ntri)) != hipSuccess ||
      hipMemcpyToSymbol(HIP_SYMBOL(c_mc_edge), edge, sizeof(edge)) != hipSuccess)
    return PIFU_ERR_HIP;
  return PIFU_OK;
}

void launch_mesh_edge_flags(const uint8_t* labels, int nn, uint8_t* flags, hipStream_t s) {
  const size_t total = (size_t)nn * nn * nn;
  hipLaunchKernelGGL(k_mesh_edge_flags, dim3(grid1d(total, 256)), dim3(256), 0, s, labels, nn, flags);
}

void launch_mesh_front(const uint8_t* labels, int nn, int32_t* kf, hipStream_t s) {
  hipLaunchKernelGGL(k_mesh_front, dim3(grid1d((size_t)nn * nn, 256)), dim3(256), 0, s, labels, nn,
                     kf);
}

void launch_mesh_verts(const uint32_t* ids, uint32_t nv, const float* occ, int nn, const int32_t* kf,
                       float* verts, uint8_t* hidden, float4* pts, hipStream_t s) {
  if (nv)
    hipLaunchKernelGGL(k_mesh_verts, dim3(grid1d(nv, 256)), dim3(256), 0, s, ids, nv, occ, nn, kf,
                       verts, hidden, pts);
}

void launch_mesh_tri_count(const uint32_t* cells, uint32_t nc, const uint8_t* labels, int nn,
                           uint32_t* cnt, hipStream_t s) {
  if (nc)
    hipLaunchKernelGGL(k_mesh_tri_count, dim3(grid1d(nc, 256)), dim3(256), 0, s, cells, nc, labels,
                       nn, cnt);
}

void launch_mesh_tri_write(const uint32_t* cells, uint32_t nc, const uint8_t* labels, int nn,
                           const uint32_t* off, const uint32_t* ids, uint32_t nv, uint32_t* tris,
                           uint32_t tri_cap, hipStream_t s) {
  if (nc)
    hipLaunchKernelGGL(k_mesh_tri_write, dim3(grid1d(nc, 256)), dim3(256), 0, s, cells, nc, labels,
                       nn, off, ids, nv, tris, tri_cap);
}

void launch_mesh_pixel_colors(const float* verts, const uint8_t* hidden, uint32_t nv,
                              const float* img, int H, int W, float* colors, hipStream_t s) {
  if (nv)
    hipLaunchKernelGGL(k_mesh_pixel_colors, dim3(grid1d(nv, 256)), dim3(256), 0, s, verts, hidden,
                       nv, img, H, W, colors);
}

}  // namespace pifu

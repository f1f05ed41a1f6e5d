// Device kernels of the particle steps around the field solve (Sec. II-A):
// point location, the exact current mapping of straight particle paths onto
// the Whitney edge functions, Faraday's update of the per-tetrahedron
// magnetic flux density, and the field interpolation + Adams-Bashforth push.
//
// Mesh data (built once per context, [nt] = tetrahedra in input order, each
// with its vertices sorted ascending so that local edge (i, j) and the
// canonical edge agree in orientation):
//   geo   [nt][12]  x_0 (vertex 0) and grad lam_1, grad lam_2, grad lam_3;
//                   lam_k(x) = g_k . (x - x_0) for k = 1..3, lam_0 = 1 - sum
//   nbr   [nt][4]   tetrahedron across the face opposite local vertex k, or -1
//   tedge [nt][6]   canonical edge of local edges 01, 02, 03, 12, 13, 23
// Particle arrays are [n][3] row-major (x, y, z per particle).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ddfem {

constexpr int kPicEdges[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

// counters of one particle launch (device, zeroed by the host before it)
enum { kPicLeftMesh = 0, kPicWalkCap = 1, kPicBadCell = 2, kPicCounters = 3 };
// longest walk of one path or location (faces crossed)
constexpr int kPicMaxCross = 1 << 16;

__global__ void __launch_bounds__(256) k_tet_geo(int64_t nt, const double* __restrict__ coords,
                                                 const int32_t* __restrict__ tsort, double* __restrict__ geo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  double x0[3], e[3][3];  // e[a] = x_{a+1} - x_0
  const int32_t v0 = tsort[4 * t];
  for (int c = 0; c < 3; ++c) x0[c] = coords[3 * (int64_t)v0 + c];
  for (int a = 0; a < 3; ++a) {
    const int32_t va = tsort[4 * t + a + 1];
    for (int c = 0; c < 3; ++c) e[a][c] = coords[3 * (int64_t)va + c] - x0[c];
  }
  // grad lam_{a+1} is the row a of the inverse of the matrix with columns
  // e[a]: g_1 = (e_2 x e_3)/det, g_2 = (e_3 x e_1)/det, g_3 = (e_1 x e_2)/det,
  // det = e_1 . (e_2 x e_3)
  double c0[3], c1[3], c2[3];
  c0[0] = e[1][1] * e[2][2] - e[1][2] * e[2][1];
  c0[1] = e[1][2] * e[2][0] - e[1][0] * e[2][2];
  c0[2] = e[1][0] * e[2][1] - e[1][1] * e[2][0];
  c1[0] = e[2][1] * e[0][2] - e[2][2] * e[0][1];
  c1[1] = e[2][2] * e[0][0] - e[2][0] * e[0][2];
  c1[2] = e[2][0] * e[0][1] - e[2][1] * e[0][0];
  c2[0] = e[0][1] * e[1][2] - e[0][2] * e[1][1];
  c2[1] = e[0][2] * e[1][0] - e[0][0] * e[1][2];
  c2[2] = e[0][0] * e[1][1] - e[0][1] * e[1][0];
  const double inv = 1.0 / (e[0][0] * c0[0] + e[0][1] * c0[1] + e[0][2] * c0[2]);
  double* o = geo + 12 * t;
  for (int c = 0; c < 3; ++c) {
    o[c] = x0[c];
    o[3 + c] = c0[c] * inv;
    o[6 + c] = c1[c] * inv;
    o[9 + c] = c2[c] * inv;
  }
}

struct PicTet {
  double x0[3], g[4][3];
};

__device__ __forceinline__ void load_tet(const double* __restrict__ geo, int64_t t, PicTet& T) {
  const double2* r = reinterpret_cast<const double2*>(geo + 12 * t);
  double v[12];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double2 u = r[i];
    v[2 * i] = u.x;
    v[2 * i + 1] = u.y;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T.x0[c] = v[c];
    T.g[1][c] = v[3 + c];
    T.g[2][c] = v[6 + c];
    T.g[3][c] = v[9 + c];
    T.g[0][c] = -(v[3 + c] + v[6 + c] + v[9 + c]);
  }
}

__device__ __forceinline__ void barycentric(const PicTet& T, const double x[3], double l[4]) {
  const double d0 = x[0] - T.x0[0], d1 = x[1] - T.x0[1], d2 = x[2] - T.x0[2];
  l[1] = T.g[1][0] * d0 + T.g[1][1] * d1 + T.g[1][2] * d2;
  l[2] = T.g[2][0] * d0 + T.g[2][1] * d1 + T.g[2][2] * d2;
  l[3] = T.g[3][0] * d0 + T.g[3][1] * d1 + T.g[3][2] * d2;
  l[0] = 1.0 - l[1] - l[2] - l[3];
}

// Exit of the straight line a -> b from tetrahedron T: in T the line is
// lam(s) = lam(a) + s (lam(b) - lam(a)); it leaves T at the smallest s where
// a decreasing lam_k reaches 0, through the face opposite k (kx = k), or not
// before s = 1 (kx = -1).
__device__ __forceinline__ void line_exit(const PicTet& T, const double a[3], const double b[3], double la[4],
                                          double d[4], double& s1, int& kx) {
  double lb[4];
  barycentric(T, a, la);
  barycentric(T, b, lb);
  // smallest la_k / -d_k over decreasing lam_k, compared as cross products
  // (denominators positive) so that only the chosen face costs a division
  double num = 1.0, den = 1.0;
  kx = -1;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    d[k] = lb[k] - la[k];
    if (d[k] < 0.0 && la[k] * den < num * -d[k]) {
      num = la[k];
      den = -d[k];
      kx = k;
    }
  }
  s1 = kx < 0 ? 1.0 : num / den;
}

// Point location: walk the straight line from the centroid of the start
// cell (cell[p], or 0 if out of range) to x[p] across shared faces.  The
// line parameter never decreases, so rounding at a face cannot send the walk
// backwards.  A line that reaches an outer face gives cell = -1.
__global__ void __launch_bounds__(256) k_pic_locate(int64_t n, int64_t nt, const double* __restrict__ x,
                                                    int32_t* __restrict__ cell, const double* __restrict__ geo,
                                                    const int32_t* __restrict__ nbr,
                                                    const double* __restrict__ coords,
                                                    const int32_t* __restrict__ tsort, int max_cross,
                                                    unsigned long long* __restrict__ cnt) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int64_t t = cell[p];
  if (t < 0 || t >= nt) t = 0;
  double a[3] = {0.0, 0.0, 0.0}, b[3];
  for (int c = 0; c < 3; ++c) b[c] = x[3 * p + c];
  for (int v = 0; v < 4; ++v) {
    const int64_t iv = tsort[4 * t + v];
    for (int c = 0; c < 3; ++c) a[c] += 0.25 * coords[3 * iv + c];
  }
  double s0 = 0.0;
  for (int it = 0;; ++it) {
    PicTet T;
    load_tet(geo, t, T);
    double la[4], d[4], s1;
    int kx;
    line_exit(T, a, b, la, d, s1, kx);
    if (kx < 0) {
      cell[p] = (int32_t)t;
      return;
    }
    s0 = s1 > s0 ? s1 : s0;
    const int32_t tn = nbr[4 * t + kx];
    if (tn < 0 || it + 1 >= max_cross) {
      cell[p] = -1;
      atomicAdd(&cnt[tn < 0 ? kPicLeftMesh : kPicWalkCap], 1ull);
      return;
    }
    t = tn;
  }
}

// Exact current mapping of the straight path xa[p] -> xb[p] (cell[p] holds
// xa[p]): the walk of k_pic_locate, and every piece [s0, s1] of the path in
// tetrahedron t adds q/dt * int W_ij . dl to the six edges of t.  On a
// straight piece lam_i dlam_j - lam_j dlam_i is constant, so with lam at s0
// and dlam = (s1 - s0)(lam(b) - lam(a)) the integral is exact.
// The contributions of a workgroup are first summed per edge in an LDS hash
// table (open addressing, kDepProbes probes, then straight to J) and the
// table is added to J with one atomic per distinct edge: with particles in
// cell order a workgroup covers a few hexahedra' worth of tetrahedra, so
// most contributions meet in LDS.  Before that, the first pieces of paths
// that start in the same cell in adjacent lanes are summed in registers.
// A path that reaches an outer face deposits up to it and the particle
// becomes inactive (cell = -1); so does a walk longer than max_cross faces.
// Inactive particles are skipped.
constexpr int kDepThreads = 512;
constexpr int kDepSlotBits = 11;
constexpr int kDepSlots = 1 << kDepSlotBits;
constexpr int kDepProbes = 16;

__device__ __forceinline__ void dep_add(int32_t* keys, double* vals, double* __restrict__ J, int32_t e, double v) {
  unsigned h = ((unsigned)e * 2654435761u) >> (32 - kDepSlotBits);
  for (int i = 0; i < kDepProbes; ++i) {
    const int32_t k = atomicCAS(&keys[h], -1, e);
    if (k == -1 || k == e) {
      atomicAdd(&vals[h], v);
      return;
    }
    h = (h + 1) & (kDepSlots - 1);
  }
  unsafeAtomicAdd(J + e, v);
}

__device__ __forceinline__ void dep_piece(int32_t* keys, double* vals, double* __restrict__ J,
                                          const int32_t* __restrict__ te, const double la[4], const double d[4],
                                          double s0, double c) {
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int i = kPicEdges[e][0], j = kPicEdges[e][1];
    const double li = la[i] + s0 * d[i], lj = la[j] + s0 * d[j];
    dep_add(keys, vals, J, te[e], c * (li * d[j] - lj * d[i]));
  }
}

__global__ void __launch_bounds__(kDepThreads) k_pic_deposit(int64_t n, int64_t nt, const double* __restrict__ xa,
                                                             const double* __restrict__ xb,
                                                             const double* __restrict__ q, double inv_dt,
                                                             int32_t* __restrict__ cell,
                                                             const double* __restrict__ geo,
                                                             const int32_t* __restrict__ nbr,
                                                             const int32_t* __restrict__ tedge,
                                                             double* __restrict__ J, int max_cross,
                                                             unsigned long long* __restrict__ cnt) {
  __shared__ int32_t keys[kDepSlots];
  __shared__ double vals[kDepSlots];
  for (int i = threadIdx.x; i < kDepSlots; i += kDepThreads) {
    keys[i] = -1;
    vals[i] = 0.0;
  }
  __syncthreads();
  const int64_t p = (int64_t)blockIdx.x * kDepThreads + threadIdx.x;
  const int lane = threadIdx.x & 63;
  int64_t t = p < n ? (int64_t)cell[p] : -1;
  if (t >= nt) {
    cell[p] = -1;
    atomicAdd(&cnt[kPicBadCell], 1ull);
    t = -1;
  }
  const bool act = t >= 0;
  // first piece (in the start cell) of every path
  double a[3], b[3], v[6], w = 0.0, s1 = 1.0;
  int kx = -1;
  if (act) {
    for (int c = 0; c < 3; ++c) {
      a[c] = xa[3 * p + c];
      b[c] = xb[3 * p + c];
    }
    w = q[p] * inv_dt;
    PicTet T;
    load_tet(geo, t, T);
    double la[4], d[4];
    line_exit(T, a, b, la, d, s1, kx);
    if (s1 < 0.0) s1 = 0.0;
    const double c = w * s1;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const int i = kPicEdges[e][0], j = kPicEdges[e][1];
      v[e] = c * (la[i] * d[j] - la[j] * d[i]);
    }
  } else {
#pragma unroll
    for (int e = 0; e < 6; ++e) v[e] = 0.0;
  }
  // runs of equal start cells in adjacent lanes (particles in cell order)
  // are summed in registers first (segmented scan; the last lane of a run
  // holds its sum), so the table sees one insert per run and edge
  const int key = act ? (int)t : -1 - lane;
  // both neighbour keys are exchanged by every lane (a shuffle inside a
  // short-circuited condition would run with its source lane switched off)
  const int kprev = __shfl_up(key, 1), knext = __shfl_down(key, 1);
  int f = (lane == 0) || (kprev != key);
  if (__any(!f)) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      double u[6];
#pragma unroll
      for (int e = 0; e < 6; ++e) u[e] = __shfl_up(v[e], off);
      const int fu = __shfl_up(f, off);
      if (lane >= off) {
        if (!f) {
#pragma unroll
          for (int e = 0; e < 6; ++e) v[e] += u[e];
        }
        f |= fu;
      }
    }
  }
  const bool tail = lane == 63 || knext != key;
  if (act) {
    if (tail) {
      const int32_t* te = tedge + 6 * t;
#pragma unroll
      for (int e = 0; e < 6; ++e) dep_add(keys, vals, J, te[e], v[e]);
    }
    // the rest of the path, piece by piece
    double s0 = s1;
    for (int it = 0; kx >= 0; ++it) {
      const int32_t tn = nbr[4 * t + kx];
      if (tn < 0 || it + 1 >= max_cross) {
        t = -1;
        atomicAdd(&cnt[tn < 0 ? kPicLeftMesh : kPicWalkCap], 1ull);
        break;
      }
      t = tn;
      PicTet T;
      load_tet(geo, t, T);
      double la[4], d[4];
      line_exit(T, a, b, la, d, s1, kx);
      if (s1 < s0) s1 = s0;
      if (s1 > s0) dep_piece(keys, vals, J, tedge + 6 * t, la, d, s0, w * (s1 - s0));
      s0 = s1;
    }
    cell[p] = (int32_t)t;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kDepSlots; i += kDepThreads) {
    const int32_t e = keys[i];
    if (e >= 0) unsafeAtomicAdd(J + e, vals[i]);
  }
}

// ---- ordering particles by cell (counting sort) -------------------------------
// count[c] (c in [0, nt], nt = inactive) -> exclusive offsets -> scatter.
// Runs of equal keys in adjacent lanes of a wavefront (particles already
// close to cell order form long runs): head and tail lane of my run.
__device__ __forceinline__ void lane_run(int key, int lane, int& head, int& tail) {
  const int kprev = __shfl_up(key, 1), knext = __shfl_down(key, 1);
  const unsigned long long heads = __ballot(lane == 0 || kprev != key);
  const unsigned long long tails = __ballot(lane == 63 || knext != key);
  head = 63 - __clzll(heads & (~0ull >> (63 - lane)));
  tail = lane + __ffsll((long long)(tails >> lane)) - 1;
}

// count[c] += number of particles in cell c (one atomic per run of a wave);
// inactive particles (cell -1 or out of range) count in c = nt
__global__ void __launch_bounds__(256) k_cell_hist(int64_t n, int64_t nt, const int32_t* __restrict__ cell,
                                                   int32_t* __restrict__ count) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  int64_t c = p < n ? (int64_t)cell[p] : -2 - lane;
  if (p < n && (c < 0 || c >= nt)) c = nt;
  int head, tail;
  lane_run((int)c, lane, head, tail);
  if (p < n && lane == tail) atomicAdd(&count[c], tail - head + 1);
}

__global__ void __launch_bounds__(256) k_zero_i32(int64_t m, int32_t* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) x[i] = 0;
}

constexpr int kScanPer = 4;                 // elements per thread
constexpr int kScanBlock = 256 * kScanPer;  // elements per workgroup

// exclusive scan of 256 values held one per thread (all 256 threads call)
__device__ __forceinline__ int block_exclusive_scan(int s, int* lds) {
  const int tid = threadIdx.x;
  lds[tid] = s;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int u = tid >= off ? lds[tid - off] : 0;
    __syncthreads();
    lds[tid] += u;
    __syncthreads();
  }
  const int incl = lds[tid];
  const int total = lds[255];
  __syncthreads();
  lds[256] = total;
  return incl - s;
}

// in place exclusive scan of each kScanBlock chunk; chunk totals to bsum
__global__ void __launch_bounds__(256) k_scan_local(int64_t m, int32_t* __restrict__ x, int32_t* __restrict__ bsum) {
  __shared__ int lds[257];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kScanPer;
  int v[kScanPer], s = 0;
  for (int j = 0; j < kScanPer; ++j) {
    v[j] = base + j < m ? x[base + j] : 0;
    s += v[j];
  }
  int run = block_exclusive_scan(s, lds);
  for (int j = 0; j < kScanPer; ++j) {
    if (base + j < m) x[base + j] = run;
    run += v[j];
  }
  if (threadIdx.x == 255) bsum[blockIdx.x] = run;
}

// in place exclusive scan of the nb chunk totals (one workgroup)
__global__ void __launch_bounds__(256) k_scan_sums(int64_t nb, int32_t* __restrict__ bsum) {
  __shared__ int lds[257];
  int carry = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += 256) {
    const int64_t i = c0 + threadIdx.x;
    const int s = i < nb ? bsum[i] : 0;
    const int ex = block_exclusive_scan(s, lds);
    if (i < nb) bsum[i] = carry + ex;
    carry += lds[256];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_scan_add(int64_t m, int32_t* __restrict__ x,
                                                  const int32_t* __restrict__ bsum) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) x[i] += bsum[i / kScanBlock];
}

__global__ void __launch_bounds__(256) k_cell_scatter(int64_t n, int64_t nt, const int32_t* __restrict__ cell,
                                                      int32_t* __restrict__ cursor, int32_t* __restrict__ perm) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  int64_t c = p < n ? (int64_t)cell[p] : -2 - lane;
  if (p < n && (c < 0 || c >= nt)) c = nt;
  int head, tail;
  lane_run((int)c, lane, head, tail);
  int base = 0;
  if (p < n && lane == tail) base = atomicAdd(&cursor[c], tail - head + 1);
  base = __shfl(base, tail);
  if (p < n) perm[base + lane - head] = (int32_t)p;
}

// dst[i] = src[perm[i]] for items of `words` 32-bit words
__global__ void __launch_bounds__(256) k_permute(int64_t n, int words, const int32_t* __restrict__ perm,
                                                 const uint32_t* __restrict__ src, uint32_t* __restrict__ dst,
                                                 unsigned long long* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * words) return;
  const int64_t r = i / words, k = i - r * words;
  const int64_t s = perm[r];
  if (s < 0 || s >= n) {
    if (k == 0) atomicAdd(&cnt[kPicBadCell], 1ull);
    return;
  }
  dst[i] = src[s * words + k];
}

// B_r[t] += alpha * curl E_r in every tetrahedron for rows r < nrows
// (E [nrows][ne], B [nrows][nt][3]), curl W_ij = 2 g_i x g_j.  The six
// curls of a tetrahedron are formed once and applied to every row.
__global__ void __launch_bounds__(256) k_pic_faraday(int64_t nt, int nrows, int64_t ne, const double* __restrict__ E,
                                                     double alpha, const double* __restrict__ geo,
                                                     const int32_t* __restrict__ tedge, double* __restrict__ B) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  PicTet T;
  load_tet(geo, t, T);
  double cw[6][3];
  int32_t ed[6];
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int i = kPicEdges[e][0], j = kPicEdges[e][1];
    ed[e] = tedge[6 * t + e];
    cw[e][0] = 2.0 * alpha * (T.g[i][1] * T.g[j][2] - T.g[i][2] * T.g[j][1]);
    cw[e][1] = 2.0 * alpha * (T.g[i][2] * T.g[j][0] - T.g[i][0] * T.g[j][2]);
    cw[e][2] = 2.0 * alpha * (T.g[i][0] * T.g[j][1] - T.g[i][1] * T.g[j][0]);
  }
  for (int r = 0; r < nrows; ++r) {
    const double* Er = E + r * ne;
    double c[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      const double f = Er[ed[e]];
      c[0] += f * cw[e][0];
      c[1] += f * cw[e][1];
      c[2] += f * cw[e][2];
    }
    double* Br = B + (r * nt + t) * 3;
    for (int k = 0; k < 3; ++k) Br[k] += c[k];
  }
}

// Field interpolation at x in its cell (E = sum_e e_e W_e, B = B[cell]) and
// one Adams-Bashforth step of x' = v, v' = (q/m)(E + v x B):
//   first: x+ = x + dt v, v+ = v + dt acc;
//   else:  x+ = x + dt (3/2 v - 1/2 v_prev), v+ = v + dt (3/2 acc - 1/2 acc_prev);
// hist [n][6] = (v_prev, acc_prev) is overwritten with (v, acc).  Inactive
// particles (cell < 0) keep x and v.
__global__ void __launch_bounds__(256) k_pic_push(int64_t n, int64_t nt, const double* __restrict__ qm,
                                                  const double* __restrict__ E, const double* __restrict__ B,
                                                  const int32_t* __restrict__ cell, const double* __restrict__ x,
                                                  double* __restrict__ xn, double* __restrict__ v,
                                                  double* __restrict__ hist, const double* __restrict__ geo,
                                                  const int32_t* __restrict__ tedge, double dt, int first,
                                                  unsigned long long* __restrict__ cnt) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t t = cell[p];
  double xp[3], vp[3];
  for (int c = 0; c < 3; ++c) {
    xp[c] = x[3 * p + c];
    vp[c] = v[3 * p + c];
  }
  if (t < 0 || t >= nt) {
    if (t >= nt) atomicAdd(&cnt[kPicBadCell], 1ull);
    for (int c = 0; c < 3; ++c) xn[3 * p + c] = xp[c];
    return;
  }
  PicTet T;
  load_tet(geo, t, T);
  double l[4];
  barycentric(T, xp, l);
  double Ef[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int i = kPicEdges[e][0], j = kPicEdges[e][1];
    const double f = E[tedge[6 * t + e]];
#pragma unroll
    for (int c = 0; c < 3; ++c) Ef[c] += f * (l[i] * T.g[j][c] - l[j] * T.g[i][c]);
  }
  const double Bx = B[3 * t], By = B[3 * t + 1], Bz = B[3 * t + 2];
  const double k = qm[p];
  double acc[3];
  acc[0] = k * (Ef[0] + vp[1] * Bz - vp[2] * By);
  acc[1] = k * (Ef[1] + vp[2] * Bx - vp[0] * Bz);
  acc[2] = k * (Ef[2] + vp[0] * By - vp[1] * Bx);
  double* h = hist + 6 * p;
  for (int c = 0; c < 3; ++c) {
    double xo, vo;
    if (first) {
      xo = xp[c] + dt * vp[c];
      vo = vp[c] + dt * acc[c];
    } else {
      xo = xp[c] + dt * (1.5 * vp[c] - 0.5 * h[c]);
      vo = vp[c] + dt * (1.5 * acc[c] - 0.5 * h[3 + c]);
    }
    h[c] = vp[c];
    h[3 + c] = acc[c];
    xn[3 * p + c] = xo;
    v[3 * p + c] = vo;
  }
}

}  // namespace ddfem

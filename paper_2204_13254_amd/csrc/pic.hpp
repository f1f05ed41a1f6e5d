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

// Walk the straight line a -> b across shared faces, starting in the
// tetrahedron that holds a.  In tetrahedron t the line is
// lam(s) = lam(a) + s (lam(b) - lam(a)); it leaves t at the smallest s where
// a decreasing lam_k reaches 0, through the face opposite k.  The parameter
// s never decreases, so rounding at a face cannot send the walk backwards.
// DEPOSIT: every piece [s0, s1] in t adds q/dt * int W_ij . dl to its six
// edges; on a straight piece lam_i dlam_j - lam_j dlam_i is constant, so
// with lam at s0 and dlam = (s1 - s0)(lam(b) - lam(a)) the integral is exact.
// A line that reaches an outer face stops there (the particle is absorbed:
// cell = -1); a walk longer than max_cross faces stops with cell = -1 too.
// Locate mode (!DEPOSIT): a is the centroid of the start cell.
template <bool DEPOSIT>
__global__ void __launch_bounds__(256) k_pic_walk(int64_t n, int64_t nt, const double* __restrict__ xa,
                                                  const double* __restrict__ xb, const double* __restrict__ q,
                                                  double inv_dt, int32_t* __restrict__ cell,
                                                  const double* __restrict__ geo, const int32_t* __restrict__ nbr,
                                                  const int32_t* __restrict__ tedge,
                                                  const double* __restrict__ coords,
                                                  const int32_t* __restrict__ tsort, double* __restrict__ J,
                                                  int max_cross, unsigned long long* __restrict__ cnt) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int64_t t = cell[p];
  double a[3], b[3];
  for (int c = 0; c < 3; ++c) b[c] = xb[3 * p + c];
  if (DEPOSIT) {
    if (t < 0) return;  // inactive particle
    if (t >= nt) {
      cell[p] = -1;
      atomicAdd(&cnt[kPicBadCell], 1ull);
      return;
    }
    for (int c = 0; c < 3; ++c) a[c] = xa[3 * p + c];
  } else {
    if (t < 0 || t >= nt) t = 0;
    for (int c = 0; c < 3; ++c) a[c] = 0.0;
    for (int v = 0; v < 4; ++v) {
      const int64_t iv = tsort[4 * t + v];
      for (int c = 0; c < 3; ++c) a[c] += 0.25 * coords[3 * iv + c];
    }
  }
  const double w = DEPOSIT ? q[p] * inv_dt : 0.0;
  double s0 = 0.0;
  for (int it = 0;; ++it) {
    PicTet T;
    load_tet(geo, t, T);
    double la[4], lb[4], d[4];
    barycentric(T, a, la);
    barycentric(T, b, lb);
    double s1 = 1.0;
    int kx = -1;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      d[k] = lb[k] - la[k];
      if (d[k] < 0.0) {
        const double s = la[k] / -d[k];
        if (s < s1) {
          s1 = s;
          kx = k;
        }
      }
    }
    if (s1 < s0) s1 = s0;
    if (DEPOSIT && s1 > s0) {
      const double c = w * (s1 - s0);
      double l[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) l[k] = la[k] + s0 * d[k];
      const int32_t* te = tedge + 6 * t;
#pragma unroll
      for (int e = 0; e < 6; ++e) {
        const int i = kPicEdges[e][0], j = kPicEdges[e][1];
        unsafeAtomicAdd(J + te[e], c * (l[i] * d[j] - l[j] * d[i]));
      }
    }
    if (kx < 0) {
      cell[p] = (int32_t)t;
      return;
    }
    s0 = s1;
    const int32_t tn = nbr[4 * t + kx];
    if (tn < 0) {
      cell[p] = -1;
      atomicAdd(&cnt[kPicLeftMesh], 1ull);
      return;
    }
    if (it + 1 >= max_cross) {
      cell[p] = -1;
      atomicAdd(&cnt[kPicWalkCap], 1ull);
      return;
    }
    t = tn;
  }
}

// B[t] += alpha * curl E in every tetrahedron, curl W_ij = 2 g_i x g_j.
__global__ void __launch_bounds__(256) k_pic_faraday(int64_t nt, const double* __restrict__ E, double alpha,
                                                     const double* __restrict__ geo,
                                                     const int32_t* __restrict__ tedge, double* __restrict__ B) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  PicTet T;
  load_tet(geo, t, T);
  double c[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    const int i = kPicEdges[e][0], j = kPicEdges[e][1];
    const double f = 2.0 * E[tedge[6 * t + e]];
    c[0] += f * (T.g[i][1] * T.g[j][2] - T.g[i][2] * T.g[j][1]);
    c[1] += f * (T.g[i][2] * T.g[j][0] - T.g[i][0] * T.g[j][2]);
    c[2] += f * (T.g[i][0] * T.g[j][1] - T.g[i][1] * T.g[j][0]);
  }
  for (int k = 0; k < 3; ++k) B[3 * t + k] += alpha * c[k];
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

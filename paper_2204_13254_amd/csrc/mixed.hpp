// Device kernels of the mixed E/B step (Sec. II-B-1: E on edges as Whitney
// 1-forms, B on faces as Whitney 2-forms), advanced by the trapezoid rule.
// Eliminating b+ = b - dt/2 C (e+ + e) from the Ampere equation leaves
//   (T + dt^2/4 S) e+ = (T - dt^2/4 S) e + dt C^T M b - dt J,
// the matrix of the decomposed solve with beta = 1/4, so the mixed step is
// one decomposed solve between a face-side right-hand side and a face
// update.  Needs the per-tetrahedron geometry of the particle tables (geo).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ddfem {

// faces of a sorted tetrahedron: the face opposite local vertex k, vertices
// ascending; and the local discrete curl C[f][e] over the local edges 01,
// 02, 03, 12, 13, 23 (boundary of face (i,j,k) = (i,j) + (j,k) - (i,k))
constexpr int kLocFaces[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
constexpr int kLocCurl[4][6] = {{0, 0, 0, 1, -1, 1}, {0, 1, -1, 0, 0, 1}, {1, 0, -1, 0, 1, 0}, {1, -1, 0, 1, 0, 0}};

// Bt[f][r] = B[r][f]: face fluxes unknown-major, so that the right-hand
// sides of one face are one contiguous line for the per-tetrahedron kernel
__global__ void __launch_bounds__(256) k_rhs_major_to_item(int64_t nf, int nrhs, const double* __restrict__ B,
                                                           double* __restrict__ Bt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf * nrhs) return;
  const int64_t f = i / nrhs;
  const int r = (int)(i - f * nrhs);
  Bt[i] = B[(int64_t)r * nf + f];
}

// out[(t*6 + a)*nrhs + r] = sum_f C[f][a] (M_t b_t)_f with M_t the 1/mu
// 2-form mass of tetrahedron t:
//   M[F][G] = (4/mu) sum_{a in F, b in G} V (1 + d_ab) / 20 c_a^F . c_b^G,
// W_F = 2 sum_{a in F} lam_a c_a^F, c_i = g_j x g_k, c_j = g_k x g_i,
// c_k = g_i x g_j for F = (i, j, k).  One thread per (tetrahedron, RHS), RHS
// fastest, so that every store of a wave fills whole lines; each RHS thread
// of a tetrahedron forms the 4x4 mass itself.  Bt is [nf][nrhs].
__global__ void __launch_bounds__(256) k_curlT_face_mass(int64_t nt, int nrhs, const double* __restrict__ Bt,
                                                         const int32_t* __restrict__ tet_faces,
                                                         const double* __restrict__ geo,
                                                         const double* __restrict__ mu, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt * nrhs) return;
  const int64_t t = i / nrhs;
  const int r = (int)(i - t * nrhs);
  PicTet T;
  load_tet(geo, t, T);
  const double(*g)[3] = T.g;
  const double det = g[1][0] * (g[2][1] * g[3][2] - g[2][2] * g[3][1]) -
                     g[1][1] * (g[2][0] * g[3][2] - g[2][2] * g[3][0]) +
                     g[1][2] * (g[2][0] * g[3][1] - g[2][1] * g[3][0]);
  const double vol = 1.0 / (6.0 * fabs(det));
  double c[4][3][3];  // c[F][m] = coefficient vector of vertex kLocFaces[F][m]
#pragma unroll
  for (int F = 0; F < 4; ++F) {
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int u = kLocFaces[F][(m + 1) % 3], v = kLocFaces[F][(m + 2) % 3];
      c[F][m][0] = g[u][1] * g[v][2] - g[u][2] * g[v][1];
      c[F][m][1] = g[u][2] * g[v][0] - g[u][0] * g[v][2];
      c[F][m][2] = g[u][0] * g[v][1] - g[u][1] * g[v][0];
    }
  }
  double b[4];
#pragma unroll
  for (int F = 0; F < 4; ++F) b[F] = Bt[(int64_t)tet_faces[4 * t + F] * nrhs + r];
  const double s = 4.0 * vol / (20.0 * mu[t]);
  double m[4];
#pragma unroll
  for (int F = 0; F < 4; ++F) {
    double acc = 0.0;
#pragma unroll
    for (int G = 0; G < 4; ++G) {
      double mfg = 0.0;
#pragma unroll
      for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double w = kLocFaces[F][p] == kLocFaces[G][k] ? 2.0 : 1.0;
          mfg += w * (c[F][p][0] * c[G][k][0] + c[F][p][1] * c[G][k][1] + c[F][p][2] * c[G][k][2]);
        }
      acc += mfg * b[G];
    }
    m[F] = s * acc;
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    double v = 0.0;
#pragma unroll
    for (int F = 0; F < 4; ++F) v += kLocCurl[F][a] * m[F];
    out[(t * 6 + a) * nrhs + r] = v;
  }
}

// y[d][r] = sum of buf over the (tet, local edge) entries of unknown d, in
// list order (a pull: no atomics, fixed order)
__global__ void __launch_bounds__(256) k_pull_edge6(int64_t nint, int nrhs, const int64_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ list, const double* __restrict__ buf,
                                                    double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nint * nrhs) return;
  const int64_t d = i / nrhs;
  const int r = (int)(i - d * nrhs);
  double s = 0.0;
  for (int64_t k = ptr[d]; k < ptr[d + 1]; ++k) s += buf[(int64_t)list[k] * nrhs + r];
  y[i] = s;
}

// right-hand side of the eliminated step: Te - (dt^2/4) Se + dt CtMb - dt J
__global__ void __launch_bounds__(256) k_mixed_rhs(int64_t n, const double* __restrict__ Te,
                                                   const double* __restrict__ Se, const double* __restrict__ cmb,
                                                   const double* __restrict__ J, double dt, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = Te[i] - 0.25 * dt * dt * Se[i] + dt * (cmb[i] - J[i]);
}

// Faraday on the faces: B+ = B - h C (E + E+), face edges fe[f] = (ab, bc, ac)
// with signs (+, +, -); all arrays RHS-major
__global__ void __launch_bounds__(256) k_face_update(int64_t nf, int nrhs, int64_t ne,
                                                     const int32_t* __restrict__ fe, const double* __restrict__ En,
                                                     const double* __restrict__ Enext, const double* __restrict__ Bn,
                                                     double* __restrict__ Bnext, double h) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nf * nrhs) return;
  const int64_t r = i / nf, f = i - r * nf;
  const double* e0 = En + r * ne;
  const double* e1 = Enext + r * ne;
  const int32_t a = fe[3 * f], b = fe[3 * f + 1], c = fe[3 * f + 2];
  const double curl = (e0[a] + e1[a]) + (e0[b] + e1[b]) - (e0[c] + e1[c]);
  Bnext[i] = Bn[i] - h * curl;
}

}  // namespace ddfem

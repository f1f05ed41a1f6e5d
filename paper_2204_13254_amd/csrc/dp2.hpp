// Device kernels of the Robin dual-primal variant (Sec. III-B, adapted to the
// edge-only system) and of its GMRES interface solver.
//
// Multipliers live per side: every interface row of every subdomain (the
// kI*NB .. kr*NB rows of its local vector, padding included) is one entry of
// a "side vector" [n_side][nrhs], in the order of those rows.  Padding rows
// are inert (code -1, no Robin row, no partner).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ddfem {

constexpr int kGmresRestart = 40;  // Krylov vectors kept before a restart

// tiles[pos[i]] += alpha * val[i]  (Robin term on the interface block, before
// the factorisation; positions are distinct)
template <class T>
__global__ void __launch_bounds__(256) k_add_entries(int64_t n, const int64_t* __restrict__ pos,
                                                     const double* __restrict__ val, double alpha,
                                                     T* __restrict__ tiles) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  tiles[pos[i]] = (T)((double)tiles[pos[i]] + alpha * val[i]);
}

// Transmission residual of the Robin condition on every side:
//   y[i] = lam[i] + lam[partner[i]] - sum_k R[i][k] u[k]
// (R = 2 alpha M_T, columns on the partner's sides), with the interface
// response u of side k read straight from its local row rows[k] of U;
// lam == nullptr gives y = -R u.
template <class T>
__global__ void __launch_bounds__(256) k_robin_apply(int64_t n, const int64_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, const double* __restrict__ val,
                                                     const int32_t* __restrict__ partner,
                                                     const double* __restrict__ lam, const int64_t* __restrict__ rows,
                                                     const T* __restrict__ U, const T* __restrict__ U2,
                                                     double* __restrict__ y, int nrhs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  const int64_t k = i / nrhs;
  const int r = (int)(i - k * nrhs);
  double s = 0.0;
  if (lam) {
    s = lam[i];
    const int32_t q = partner[k];
    if (q >= 0) s += lam[(int64_t)q * nrhs + r];
  }
  for (int64_t j = rp[k]; j < rp[k + 1]; ++j) {
    const int64_t x = rows[ci[j]] * nrhs + r;
    const T u = U2 ? (T)(U[x] + U2[x]) : U[x];
    s -= val[j] * (double)u;
  }
  y[i] = s;
}

// Block shares of nv dot products V_k . w per right-hand side:
// partial[(k * gridDim.x + b) * kMaxRhs + r] (fixed order, no atomics).
// Workgroup row y takes vectors 8y .. 8y+7, so w is read once per 8 vectors.
constexpr int kMdotChunk = 8;

__global__ void __launch_bounds__(256) k_mdot(int64_t n, int nv, const double* __restrict__ V, int64_t ldv,
                                              const double* __restrict__ w, int nrhs, double* __restrict__ partial) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int lpr = 256 / nrhs;
  const int r = tid % nrhs, lane = tid / nrhs;
  const int k0 = blockIdx.y * kMdotChunk;
  const int kn = nv - k0 < kMdotChunk ? nv - k0 : kMdotChunk;
  double s[kMdotChunk];
#pragma unroll
  for (int k = 0; k < kMdotChunk; ++k) s[k] = 0.0;
  if (lane < lpr)
    for (int64_t row = (int64_t)blockIdx.x * lpr + lane; row < n; row += (int64_t)gridDim.x * lpr) {
      const int64_t e = row * nrhs + r;
      const double x = w[e];
#pragma unroll
      for (int k = 0; k < kMdotChunk; ++k)
        if (k < kn) s[k] += V[(k0 + k) * ldv + e] * x;
    }
#pragma unroll
  for (int k = 0; k < kMdotChunk; ++k) {
    if (k >= kn) break;
    red[tid] = s[k];
    __syncthreads();
    if (tid < nrhs) {
      double t = 0.0;
      for (int l = 0; l < lpr; ++l) t += red[l * nrhs + tid];
      partial[((int64_t)(k0 + k) * gridDim.x + blockIdx.x) * kMaxRhs + tid] = t;
    }
    __syncthreads();
  }
}

// h[k][r] = sum_b partial (fixed order); tot[k][r] += h[k][r] if tot.  One
// workgroup per k: a power-of-two number of lanes per right-hand side take
// strided block shares, then a fixed-shape tree in LDS.
__global__ void __launch_bounds__(256) k_mdot_reduce(int nv, int nrhs, int nblocks, const double* __restrict__ partial,
                                                     double* __restrict__ h, double* __restrict__ tot) {
  __shared__ double red[256];
  const int k = blockIdx.x;
  const int tid = threadIdx.x;
  int lpr = 1;  // lanes per right-hand side: a power of two, so the tree halves evenly
  while (2 * lpr * nrhs <= 256) lpr *= 2;
  const int r = tid % nrhs, lane = tid / nrhs;
  double s = 0.0;
  if (lane < lpr)
    for (int b = lane; b < nblocks; b += lpr) s += partial[((int64_t)k * nblocks + b) * kMaxRhs + r];
  red[tid] = s;
  __syncthreads();
  for (int half = lpr / 2; half > 0; half /= 2) {
    if (lane < half) red[tid] += red[tid + half * nrhs];
    __syncthreads();
  }
  if (tid < nrhs) {
    h[k * kMaxRhs + tid] = red[tid];
    if (tot) tot[k * kMaxRhs + tid] += red[tid];
  }
}

// w[i][r] += sgn * sum_k h[k][r] V_k[i][r]
__global__ void __launch_bounds__(256) k_mupdate(int64_t n, int nv, const double* __restrict__ V, int64_t ldv,
                                                 const double* __restrict__ h, double sgn, double* __restrict__ w,
                                                 int nrhs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  const int r = (int)(i % nrhs);
  double s = 0.0;
  for (int k = 0; k < nv; ++k) s += h[k * kMaxRhs + r] * V[k * ldv + i];
  w[i] += sgn * s;
}

// y = a - y in place (restart residual: y holds G lam on entry)
__global__ void __launch_bounds__(256) k_rsub(int64_t n, const double* __restrict__ a, double* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a[i] - y[i];
}

// out = w / sqrt(ss[r]) per right-hand side (0 where ss is not positive)
__global__ void __launch_bounds__(256) k_vnormalize(int64_t n, const double* w, const double* __restrict__ ss,
                                                    double* out, int nrhs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  const double q = ss[i % nrhs];
  out[i] = q > 0.0 ? w[i] / sqrt(q) : 0.0;
}

}  // namespace ddfem

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
// response u of side k read straight from its local row rrow[j] of U (the
// row of column j, resolved at setup); lam == nullptr gives y = -R u.
template <class T>
__global__ void __launch_bounds__(256) k_robin_apply(int64_t n, const int64_t* __restrict__ rp,
                                                     const int64_t* __restrict__ rrow, const double* __restrict__ val,
                                                     const int32_t* __restrict__ partner,
                                                     const double* __restrict__ lam, const T* __restrict__ U,
                                                     const T* __restrict__ U2, double* __restrict__ y, int nrhs,
                                                     const int* __restrict__ skip) {
  if (skip && *skip) return;
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
  const int64_t j0 = rp[k], j1 = rp[k + 1];
  for (int64_t j = j0; j < j1; ++j) {
    const int64_t x = rrow[j] * nrhs + r;
    const T u = U2 ? (T)(U[x] + U2[x]) : U[x];
    s -= val[j] * (double)u;
  }
  y[i] = s;
}

// Vector form of k_robin_apply: one thread per (side row, group of V
// right-hand sides), each gather one load of V consecutive values (nrhs a
// multiple of V); the same sums in the same order.
template <class T, int V>
__global__ void __launch_bounds__(256) k_robin_apply_v(int64_t n, const int64_t* __restrict__ rp,
                                                       const int64_t* __restrict__ rrow,
                                                       const double* __restrict__ val,
                                                       const int32_t* __restrict__ partner,
                                                       const double* __restrict__ lam, const T* __restrict__ U,
                                                       const T* __restrict__ U2, double* __restrict__ y, int nrhs,
                                                       const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int G = nrhs / V;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * G) return;
  const int64_t k = i / G;
  const int q = (int)(i - k * G);
  double s[V];
  if (lam) {
    vload<double, V>(lam + k * nrhs + q * V, s);
    const int32_t pq = partner[k];
    if (pq >= 0) {
      double t[V];
      vload<double, V>(lam + (int64_t)pq * nrhs + q * V, t);
#pragma unroll
      for (int w = 0; w < V; ++w) s[w] += t[w];
    }
  } else {
#pragma unroll
    for (int w = 0; w < V; ++w) s[w] = 0.0;
  }
  const int64_t j0 = rp[k], j1 = rp[k + 1];
  for (int64_t j = j0; j < j1; ++j) {
    const int64_t x = rrow[j] * nrhs + q * V;
    T u[V];
    vload<T, V>(U + x, u);
    if (U2) {
      T u2[V];
      vload<T, V>(U2 + x, u2);
#pragma unroll
      for (int w = 0; w < V; ++w) u[w] = (T)(u[w] + u2[w]);
    }
    const double a = val[j];
#pragma unroll
    for (int w = 0; w < V; ++w) s[w] -= a * (double)u[w];
  }
  vstore<double, V>(y + k * nrhs + q * V, s);
}

// Block shares of nv dot products V_k . w per right-hand side:
// partial[(k * gridDim.x + b) * kMaxRhs + r] (fixed order, no atomics).
// Workgroup row y takes vectors 8y .. 8y+7, so w is read once per 8 vectors.
constexpr int kMdotChunk = 8;

__global__ void __launch_bounds__(256) k_mdot(int64_t n, int nv, const double* __restrict__ V, int64_t ldv,
                                              const double* __restrict__ w, int nrhs, double* __restrict__ partial,
                                              const int* __restrict__ skip) {
  if (skip && *skip) return;
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

// Vector form of k_mdot: V right-hand sides per lane (nrhs a multiple of
// V), one 8V-byte load of each vector per row.
template <int V>
__global__ void __launch_bounds__(256) k_mdot_v(int64_t n, int nv, const double* __restrict__ Vb, int64_t ldv,
                                                const double* __restrict__ w, int nrhs, double* __restrict__ partial,
                                                const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int tid = threadIdx.x;
  const int G = nrhs / V, lpr = 256 / G;
  const int q = tid % G, lane = tid / G;
  const int k0 = blockIdx.y * kMdotChunk;
  const int kn = nv - k0 < kMdotChunk ? nv - k0 : kMdotChunk;
  double s[kMdotChunk][V];
#pragma unroll
  for (int k = 0; k < kMdotChunk; ++k)
#pragma unroll
    for (int u = 0; u < V; ++u) s[k][u] = 0.0;
  if (lane < lpr)
    for (int64_t row = (int64_t)blockIdx.x * lpr + lane; row < n; row += (int64_t)gridDim.x * lpr) {
      const int64_t e = row * nrhs + q * V;
      double x[V];
      vload<double, V>(w + e, x);
#pragma unroll
      for (int k = 0; k < kMdotChunk; ++k)
        if (k < kn) {
          double a[V];
          vload<double, V>(Vb + (k0 + k) * ldv + e, a);
#pragma unroll
          for (int u = 0; u < V; ++u) s[k][u] += a[u] * x[u];
        }
    }
  __shared__ double red[256 * V];
#pragma unroll
  for (int k = 0; k < kMdotChunk; ++k) {
    if (k >= kn) break;
#pragma unroll
    for (int u = 0; u < V; ++u) red[tid * V + u] = s[k][u];
    __syncthreads();
    if (tid < nrhs) {
      const int qq = tid / V, u = tid % V;
      double t = 0.0;
      for (int l = 0; l < lpr; ++l) t += red[(l * G + qq) * V + u];
      partial[((int64_t)(k0 + k) * gridDim.x + blockIdx.x) * kMaxRhs + tid] = t;
    }
    __syncthreads();
  }
}

// h[k][r] = sum_b partial (fixed order); with tot, tot[k][r] = h[k][r]
// (assign) or tot[k][r] += h[k][r].  One workgroup per k: a power-of-two
// number of lanes per right-hand side take strided block shares, then a
// fixed-shape tree in LDS.
__global__ void __launch_bounds__(256) k_mdot_reduce(int nv, int nrhs, int nblocks, const double* __restrict__ partial,
                                                     double* __restrict__ h, double* __restrict__ tot, int assign,
                                                     const int* __restrict__ skip) {
  if (skip && *skip) return;
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
    if (tot) tot[k * kMaxRhs + tid] = assign ? red[tid] : tot[k * kMaxRhs + tid] + red[tid];
  }
}

// w[i][r] += sgn * sum_k h[k][r] V_k[i][r] over k < nv, or k < *nvp when
// nvp is given (a count the device decided)
__global__ void __launch_bounds__(256) k_mupdate(int64_t n, int nv, const double* __restrict__ V, int64_t ldv,
                                                 const double* __restrict__ h, double sgn, double* __restrict__ w,
                                                 int nrhs, const int* __restrict__ nvp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  if (nvp) nv = *nvp;
  const int r = (int)(i % nrhs);
  double s = 0.0;
  for (int k = 0; k < nv; ++k) s += h[k * kMaxRhs + r] * V[k * ldv + i];
  w[i] += sgn * s;
}

// The two projections of classical Gram-Schmidt applied twice on the new
// vector w = V_{j+1} against the basis V_0 .. V_j (nv = j + 1 vectors, nv <=
// KMAX), each one pass over the basis.  Grid-stride over rows (layout
// [n][nrhs]), kDotBlocks workgroups; the coefficients h [k][kMaxRhs] are
// staged in LDS.
//  first:  w' = w - sum_k h1_k V_k, with the block partials of V_k . w' (k <
//          nv) and of |w'|^2 (index nv), for the second projection
//  second: w'' = (w' - sum_k h2_k V_k) / sqrt(ss) (ss from k_gm_givens; 0
//          where ss is not positive)
template <int KMAX, bool FIRST>
__global__ void __launch_bounds__(256) k_gm_project(int64_t n, int nv, const double* __restrict__ V, int64_t ldv,
                                                    const double* __restrict__ h, double* __restrict__ w, int nrhs,
                                                    double* __restrict__ partial, const double* __restrict__ ss,
                                                    const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double hs[KMAX * kMaxRhs];
  __shared__ double red[256];
  for (int t = threadIdx.x; t < nv * kMaxRhs; t += blockDim.x) hs[t] = h[t];
  __syncthreads();
  const int lpr = 256 / nrhs;
  const int tid = threadIdx.x, r = tid % nrhs, lane = tid / nrhs;
  double hk[KMAX], dots[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    hk[k] = k < nv ? hs[k * kMaxRhs + r] : 0.0;
    dots[k] = 0.0;
  }
  double nn = 0.0;
  double scale = 1.0;
  if (!FIRST) {
    const double q = ss[r];
    scale = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
  }
  if (lane < lpr)
    for (int64_t row = (int64_t)blockIdx.x * lpr + lane; row < n; row += (int64_t)gridDim.x * lpr) {
      const int64_t e = row * nrhs + r;
      double vk[KMAX];
#pragma unroll
      for (int k = 0; k < KMAX; ++k) vk[k] = k < nv ? V[k * ldv + e] : 0.0;
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < KMAX; ++k) acc += hk[k] * vk[k];
      const double v = w[e] - acc;
      if (FIRST) {
        w[e] = v;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) dots[k] += vk[k] * v;
        nn += v * v;
      } else {
        w[e] = v * scale;
      }
    }
  if (!FIRST) return;
  // block partials of the nv dots and |w'|^2 (fixed order)
#pragma unroll
  for (int k = 0; k <= KMAX; ++k) {
    if (k > nv) break;
    red[tid] = k < nv ? dots[k < KMAX ? k : 0] : nn;
    __syncthreads();
    if (tid < nrhs) {
      double t = 0.0;
      for (int l2 = 0; l2 < lpr; ++l2) t += red[l2 * nrhs + tid];
      partial[((int64_t)k * gridDim.x + blockIdx.x) * kMaxRhs + tid] = t;
    }
    __syncthreads();
  }
}

// Vector form of k_gm_project: V right-hand sides per lane (nrhs a multiple
// of V); the same sums per right-hand side.
template <int KMAX, bool FIRST, int V>
__global__ void __launch_bounds__(256) k_gm_project_v(int64_t n, int nv, const double* __restrict__ Vb, int64_t ldv,
                                                      const double* __restrict__ h, double* __restrict__ w, int nrhs,
                                                      double* __restrict__ partial, const double* __restrict__ ss,
                                                      const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double hs[KMAX * kMaxRhs];
  __shared__ double red[256 * V];
  for (int t = threadIdx.x; t < nv * kMaxRhs; t += blockDim.x) hs[t] = h[t];
  __syncthreads();
  const int G = nrhs / V, lpr = 256 / G;
  const int tid = threadIdx.x, q = tid % G, lane = tid / G;
  double hk[KMAX][V], dots[KMAX][V];
#pragma unroll
  for (int k = 0; k < KMAX; ++k)
#pragma unroll
    for (int u = 0; u < V; ++u) {
      hk[k][u] = k < nv ? hs[k * kMaxRhs + q * V + u] : 0.0;
      dots[k][u] = 0.0;
    }
  double nn[V], scale[V];
#pragma unroll
  for (int u = 0; u < V; ++u) {
    nn[u] = 0.0;
    scale[u] = 1.0;
    if (!FIRST) {
      const double qq = ss[q * V + u];
      scale[u] = qq > 0.0 ? 1.0 / sqrt(qq) : 0.0;
    }
  }
  if (lane < lpr)
    for (int64_t row = (int64_t)blockIdx.x * lpr + lane; row < n; row += (int64_t)gridDim.x * lpr) {
      const int64_t e = row * nrhs + q * V;
      double vk[KMAX][V];
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k < nv) {
          vload<double, V>(Vb + k * ldv + e, vk[k]);
        } else {
#pragma unroll
          for (int u = 0; u < V; ++u) vk[k][u] = 0.0;
        }
      }
      double wv[V];
      vload<double, V>(w + e, wv);
#pragma unroll
      for (int u = 0; u < V; ++u) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < KMAX; ++k) acc += hk[k][u] * vk[k][u];
        const double v = wv[u] - acc;
        if (FIRST) {
          wv[u] = v;
#pragma unroll
          for (int k = 0; k < KMAX; ++k) dots[k][u] += vk[k][u] * v;
          nn[u] += v * v;
        } else {
          wv[u] = v * scale[u];
        }
      }
      vstore<double, V>(w + e, wv);
    }
  if (!FIRST) return;
  // block partials of the nv dots and |w'|^2 (fixed order)
#pragma unroll
  for (int k = 0; k <= KMAX; ++k) {
    if (k > nv) break;
#pragma unroll
    for (int u = 0; u < V; ++u) red[tid * V + u] = k < nv ? dots[k < KMAX ? k : 0][u] : nn[u];
    __syncthreads();
    if (tid < nrhs) {
      const int qq = tid / V, u = tid % V;
      double t = 0.0;
      for (int l2 = 0; l2 < lpr; ++l2) t += red[(l2 * G + qq) * V + u];
      partial[((int64_t)k * gridDim.x + blockIdx.x) * kMaxRhs + tid] = t;
    }
    __syncthreads();
  }
}

// y = a - y in place (restart residual: y holds G lam on entry)
__global__ void __launch_bounds__(256) k_rsub(int64_t n, const double* __restrict__ a, double* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a[i] - y[i];
}

// out = w / sqrt(ss[r]) per right-hand side (0 where ss is not positive)
__global__ void __launch_bounds__(256) k_vnormalize(int64_t n, const double* w, const double* __restrict__ ss,
                                                    double* out, int nrhs, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  const double q = ss[i % nrhs];
  out[i] = q > 0.0 ? w[i] / sqrt(q) : 0.0;
}

// ---------------------------------------------------------------------------
// GMRES scalar work on the device.  The Hessenberg columns, the Givens
// rotations and the least-squares right-hand side of every RHS stay in
// device memory; small single-workgroup kernels advance them, so an
// iteration needs no host round trip and a block of iterations replays as
// one captured graph.  Every RHS iterates in lock step; a converged RHS
// keeps its columns and stops updating them.
// ---------------------------------------------------------------------------
struct GmState {
  double bnorm[kMaxRhs];   // |rhs|
  double relres[kMaxRhs];  // |g_{j+1}| / |rhs| after the RHS's last iteration
  double ss[kMaxRhs];      // |w|^2 of the newest basis vector (its normaliser)
  int conv[kMaxRhs];
  int cols[kMaxRhs];       // Hessenberg columns of the current cycle
  int iters[kMaxRhs];      // iterations of the whole solve
  int total;               // iterations launched that did work
  int stop;                // every RHS converged or the cap reached: gate of the iteration kernels
  int jmax;                // columns of the cycle's update (the largest cols)
};

// fixed-order total of kDotBlocks block partials ([kDotBlocks][kMaxRhs]) of
// right-hand side threadIdx.x (valid for threadIdx.x < nrhs) by a workgroup
// of kScalarThreads threads
__device__ __forceinline__ double gm_total(const double* __restrict__ pa, int nrhs, double* part) {
  const int t = threadIdx.x, lpr = blockDim.x / nrhs, rr = t % nrhs, ln = t / nrhs;
  double a = 0.0;
  if (ln < lpr)
    for (int b = ln; b < kDotBlocks; b += lpr) a += pa[b * kMaxRhs + rr];
  part[t] = a;
  __syncthreads();
  double v = 0.0;
  if (t < nrhs)
    for (int l = 0; l < lpr; ++l) v += part[l * nrhs + t];
  __syncthreads();
  return v;
}

// start of the solve: partial = block partials of |rhs|^2
__global__ void __launch_bounds__(kScalarThreads) k_gm_init(int nrhs, const double* __restrict__ partial,
                                                            GmState* __restrict__ st) {
  __shared__ double part[kScalarThreads];
  __shared__ int any_open;
  if (threadIdx.x == 0) any_open = 0;
  const double s = gm_total(partial, nrhs, part);
  const int r = threadIdx.x;
  if (r < nrhs) {
    const double b = sqrt(s > 0.0 ? s : 0.0);
    st->bnorm[r] = b;
    st->conv[r] = b > 0.0 ? 0 : 1;
    st->relres[r] = 0.0;
    st->iters[r] = 0;
    st->cols[r] = 0;
    if (!st->conv[r]) atomicOr(&any_open, 1);
  }
  __syncthreads();
  if (r == 0) {
    st->total = 0;
    st->stop = any_open ? 0 : 1;
    st->jmax = 0;
  }
}

// start of a restart cycle: partial = block partials of |r0|^2; g = |r0| e_1
__global__ void __launch_bounds__(kScalarThreads) k_gm_cycle(int nrhs, const double* __restrict__ partial,
                                                             GmState* __restrict__ st, double* __restrict__ g, int m,
                                                             int cap) {
  __shared__ double part[kScalarThreads];
  __shared__ int any_open;
  if (threadIdx.x == 0) any_open = 0;
  const double s = gm_total(partial, nrhs, part);
  const int r = threadIdx.x;
  if (r < nrhs) {
    st->ss[r] = s;
    st->cols[r] = 0;
    double* gr = g + (int64_t)r * (m + 1);
    gr[0] = sqrt(s > 0.0 ? s : 0.0);
    for (int i = 1; i <= m; ++i) gr[i] = 0.0;
    if (!st->conv[r]) atomicOr(&any_open, 1);
  }
  __syncthreads();
  if (r == 0) {
    st->stop = (any_open && st->total < cap) ? 0 : 1;
  }
}

// End of iteration j, after the two projections of classical Gram-Schmidt:
// tot[0..j] = h1 + h2, the column of the Hessenberg matrix above its
// subdiagonal; h2[0..j] = the second projection's coefficients and h2[j+1]
// = |w'|^2 after the first projection, so |w''|^2 = |w'|^2 - |h2|^2 (w' - V
// h2 is orthogonal to the basis; clamped at 0).  Per open RHS: apply the
// earlier rotations to the column, form the new one, rotate g, test
// |g_{j+1}|.  ss = |w''|^2 normalises the new basis vector.
// H: [nrhs][m][m+1] (column-major per RHS), cs/sn: [nrhs][m], g: [nrhs][m+1].
__global__ void __launch_bounds__(kScalarThreads) k_gm_givens(int j, int nrhs, const double* __restrict__ h2,
                                                              const double* __restrict__ tot, GmState* __restrict__ st,
                                                              double* __restrict__ H, double* __restrict__ cs,
                                                              double* __restrict__ sn, double* __restrict__ g, int m,
                                                              double tol, int cap, const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ int any_open;
  if (threadIdx.x == 0) any_open = 0;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x < nrhs) {
    const int rr = threadIdx.x;
    double p = 0.0;
    for (int k = 0; k <= j; ++k) p += h2[k * kMaxRhs + rr] * h2[k * kMaxRhs + rr];
    s = h2[(j + 1) * kMaxRhs + rr] - p;
    s = s > 0.0 ? s : 0.0;
  }
  const int r = threadIdx.x;
  if (r < nrhs) {
    st->ss[r] = s;
    if (!st->conv[r]) {
      double* h = H + ((int64_t)r * m + j) * (m + 1);
      for (int i = 0; i <= j; ++i) h[i] = tot[i * kMaxRhs + r];
      h[j + 1] = sqrt(s > 0.0 ? s : 0.0);
      double* c = cs + (int64_t)r * m;
      double* sv = sn + (int64_t)r * m;
      for (int i = 0; i < j; ++i) {
        const double a = h[i], b = h[i + 1];
        h[i] = c[i] * a + sv[i] * b;
        h[i + 1] = -sv[i] * a + c[i] * b;
      }
      const double d = hypot(h[j], h[j + 1]);
      c[j] = d > 0.0 ? h[j] / d : 1.0;
      sv[j] = d > 0.0 ? h[j + 1] / d : 0.0;
      h[j] = d;
      h[j + 1] = 0.0;
      double* gr = g + (int64_t)r * (m + 1);
      gr[j + 1] = -sv[j] * gr[j];
      gr[j] = c[j] * gr[j];
      st->cols[r] = j + 1;
      st->iters[r] += 1;
      const double rel = fabs(gr[j + 1]) / st->bnorm[r];
      st->relres[r] = rel;
      if (rel <= tol) st->conv[r] = 1;
    }
    if (!st->conv[r]) atomicOr(&any_open, 1);
  }
  __syncthreads();
  if (r == 0) {
    const int total = st->total + 1;
    st->total = total;
    if (!any_open || total >= cap) st->stop = 1;
  }
}

// End of a cycle: y = R^-1 g over each RHS's first cols columns (zero
// beyond), y: [m][kMaxRhs]; jmax = the largest cols
__global__ void __launch_bounds__(kScalarThreads) k_gm_solve(int nrhs, GmState* __restrict__ st,
                                                             const double* __restrict__ H, const double* __restrict__ g,
                                                             double* __restrict__ y, int m) {
  __shared__ int jmax;
  if (threadIdx.x == 0) jmax = 0;
  __syncthreads();
  const int r = threadIdx.x;
  if (r < nrhs) {
    const int k = st->cols[r];
    const double* gr = g + (int64_t)r * (m + 1);
    for (int i = m - 1; i >= k; --i) y[i * kMaxRhs + r] = 0.0;
    for (int i = k - 1; i >= 0; --i) {
      double v = gr[i];
      for (int q = i + 1; q < k; ++q) v -= H[((int64_t)r * m + q) * (m + 1) + i] * y[q * kMaxRhs + r];
      const double diag = H[((int64_t)r * m + i) * (m + 1) + i];
      y[i * kMaxRhs + r] = diag != 0.0 ? v / diag : 0.0;
    }
    atomicMax(&jmax, k);
  }
  __syncthreads();
  if (r == 0) st->jmax = jmax;
}

}  // namespace ddfem

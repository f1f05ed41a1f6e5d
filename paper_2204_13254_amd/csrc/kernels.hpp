// Device kernels of the domain-decomposed Newmark solve (gfx950, wave64).
//
// Storage: every dense per-subdomain matrix (and the coarse corner matrix)
// is a packed lower triangle of NB x NB tiles, tile (i, j), i >= j, at
// tile index tile_off + i(i+1)/2 + j, each tile row-major.  Local vectors
// are [rows][nrhs] row-major with rows = K*NB per subdomain.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ddfem {

constexpr int kNB = 32;
constexpr int kTile = kNB * kNB;
constexpr int kMaxRhs = 32;

struct SubDev {
  int32_t nI, nG, nC;
  int32_t kI, kG, kC, K;
  int32_t pad_;
  int64_t tile_off;
  int64_t row_off;
};

__device__ __forceinline__ int64_t tile_index(const SubDev& q, int i, int j) {
  return q.tile_off + (int64_t)i * (i + 1) / 2 + j;
}

// 16x16x4 MFMA (f32 / f64).  Operands (checked on the device): lane l gives
// A[l%16][l/16] and B[l/16][l%16]; accumulator element v of lane l is
// D[row(l, v)][l%16], with row = 4(l/16) + v for f32 and l/16 + 4v for f64.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <class T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef f32x4 acc_t;
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output row (within the 16-row block) of accumulator element v of lane l
  static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};
template <>
struct Mfma<double> {
  typedef f64x4 acc_t;
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
};

// One wave's 16x16 block (mb, nb) of a 32x32 tile product from LDS tiles:
// BT ? A B^T : A B, accumulated into acc.
template <class T, bool BT>
__device__ __forceinline__ void tile_mma(const T (*A)[kNB + 1], const T (*B)[kNB + 1], int mb, int nb, int l,
                                         typename Mfma<T>::acc_t& acc) {
  const int i = l & 15, g = l >> 4;
#pragma unroll
  for (int ks = 0; ks < kNB / 4; ++ks) {
    const T a = A[mb * 16 + i][ks * 4 + g];
    const T b = BT ? B[nb * 16 + i][ks * 4 + g] : B[ks * 4 + g][nb * 16 + i];
    acc = Mfma<T>::op(a, b, acc);
  }
}

// List, in increasing order, of the m in [m0, m1) with ok(m), built by the
// whole 256-thread workgroup with ballots (list holds m1 - m0 entries, m1 <=
// 65536); returns the count.  Every thread must call it.
template <class Ok>
__device__ __forceinline__ int chain_list(int m0, int m1, Ok ok, uint16_t* list, int* wcnt) {
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  int nn = 0;
  for (int b0 = m0; b0 < m1; b0 += 256) {
    const int m = b0 + tid;
    const bool nz = m < m1 && ok(m);
    const unsigned long long bal = __ballot(nz);
    if (l == 0) wcnt[w] = __popcll(bal);
    __syncthreads();
    int off = nn;
    for (int x = 0; x < w; ++x) off += wcnt[x];
    if (nz) list[off + __popcll(bal & ((1ull << l) - 1ull))] = (uint16_t)m;
    nn += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    __syncthreads();
  }
  return nn;
}

// acc += sum over the listed m of A_m B_m (B_m^T with BT; A_m staged
// transposed with AT), ptr(m, a, b) giving the two tiles.  The next term's
// tiles are loaded into registers while the current product runs.
template <class T, bool AT, bool BT, class Ptr>
__device__ __forceinline__ void chain_mma(const uint16_t* list, int nn, Ptr ptr, T (*A)[kNB + 1],
                                          T (*B)[kNB + 1], typename Mfma<T>::acc_t& acc) {
  constexpr int E = kTile / 256;
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, mb = w >> 1, nb = w & 1;
  if (nn == 0) return;
  T ra[E], rb[E];
  const T* ap;
  const T* bp;
  ptr((int)list[0], ap, bp);
#pragma unroll
  for (int u = 0; u < E; ++u) {
    ra[u] = ap[tid + 256 * u];
    rb[u] = bp[tid + 256 * u];
  }
  for (int t = 0; t < nn; ++t) {
    __syncthreads();  // the previous product has read A and B
#pragma unroll
    for (int u = 0; u < E; ++u) {
      const int e = tid + 256 * u;
      if (AT) A[e % kNB][e / kNB] = ra[u];
      else A[e / kNB][e % kNB] = ra[u];
      B[e / kNB][e % kNB] = rb[u];
    }
    __syncthreads();
    if (t + 1 < nn) {
      ptr((int)list[t + 1], ap, bp);
#pragma unroll
      for (int u = 0; u < E; ++u) {
        ra[u] = ap[tid + 256 * u];
        rb[u] = bp[tid + 256 * u];
      }
    }
    tile_mma<T, BT>(A, B, mb, nb, l, acc);
  }
}

// --------------------------------------------------------------------------
// K1: element matrices (Sec. II-B-1, Whitney 1-forms), FP64.
// Te[(ij),(kl)] = eps V/20 [(1+d_ik) g_j.g_l - (1+d_il) g_j.g_k
//                          - (1+d_jk) g_i.g_l + (1+d_jl) g_i.g_k]
// Se[(ij),(kl)] = (4V/mu) (g_i x g_j).(g_k x g_l)
// with g = grad(barycentric), local edges 01,02,03,12,13,23 of the sorted
// tetrahedron.  Te is stored with eps = 1 (unit mass) and scaled where used.
// --------------------------------------------------------------------------
__global__ void k_element(int64_t nt, const double* __restrict__ coords,
                          const int32_t* __restrict__ tsort, const double* __restrict__ mu,
                          double* __restrict__ Te, double* __restrict__ Se) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  double x[4][3];
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 3; ++c) x[a][c] = coords[3 * (int64_t)tsort[4 * t + a] + c];
  double d[3][3];
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) d[a][c] = x[a + 1][c] - x[0][c];
  // rows of inverse of D (D has columns d[a]) are grad lam_1..3:
  // inv(D) = adj(D)/det, with D[c][a] = d[a][c]
  double D[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) D[r][c] = d[c][r];
  double det = D[0][0] * (D[1][1] * D[2][2] - D[1][2] * D[2][1]) -
               D[0][1] * (D[1][0] * D[2][2] - D[1][2] * D[2][0]) +
               D[0][2] * (D[1][0] * D[2][1] - D[1][1] * D[2][0]);
  double inv = 1.0 / det;
  double g[4][3];
  g[1][0] = (D[1][1] * D[2][2] - D[1][2] * D[2][1]) * inv;
  g[1][1] = (D[0][2] * D[2][1] - D[0][1] * D[2][2]) * inv;
  g[1][2] = (D[0][1] * D[1][2] - D[0][2] * D[1][1]) * inv;
  g[2][0] = (D[1][2] * D[2][0] - D[1][0] * D[2][2]) * inv;
  g[2][1] = (D[0][0] * D[2][2] - D[0][2] * D[2][0]) * inv;
  g[2][2] = (D[0][2] * D[1][0] - D[0][0] * D[1][2]) * inv;
  g[3][0] = (D[1][0] * D[2][1] - D[1][1] * D[2][0]) * inv;
  g[3][1] = (D[0][1] * D[2][0] - D[0][0] * D[2][1]) * inv;
  g[3][2] = (D[0][0] * D[1][1] - D[0][1] * D[1][0]) * inv;
  for (int c = 0; c < 3; ++c) g[0][c] = -(g[1][c] + g[2][c] + g[3][c]);
  double V = fabs(det) / 6.0;
  double gg[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) gg[a][b] = g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2];
  const int LE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  double cr[6][3];
  for (int e = 0; e < 6; ++e) {
    const double* u = g[LE[e][0]];
    const double* v = g[LE[e][1]];
    cr[e][0] = u[1] * v[2] - u[2] * v[1];
    cr[e][1] = u[2] * v[0] - u[0] * v[2];
    cr[e][2] = u[0] * v[1] - u[1] * v[0];
  }
  double m = V / 20.0, sc = 4.0 * V / mu[t];
  for (int A = 0; A < 6; ++A) {
    int i = LE[A][0], j = LE[A][1];
    for (int B = 0; B < 6; ++B) {
      int k = LE[B][0], l = LE[B][1];
      double te = (1 + (i == k)) * gg[j][l] - (1 + (i == l)) * gg[j][k] - (1 + (j == k)) * gg[i][l] +
                  (1 + (j == l)) * gg[i][k];
      Te[36 * t + 6 * A + B] = m * te;
      Se[36 * t + 6 * A + B] = sc * (cr[A][0] * cr[B][0] + cr[A][1] * cr[B][1] + cr[A][2] * cr[B][2]);
    }
  }
}

// Pull assembly into the per-subdomain tile stores: entry e sums its
// contributions c in [ptr[e], ptr[e+1]) (contribution = tet*36 + a*6 + b)
// in a fixed order in FP64, then writes once (deterministic, no atomics).
// A = eps T_unit + cs * S.
template <class T>
__global__ void k_pull_local(int64_t n_entries, const int64_t* __restrict__ ptr,
                             const int32_t* __restrict__ contrib, const int64_t* __restrict__ dest,
                             const double* __restrict__ Te, const double* __restrict__ Se,
                             const double* __restrict__ eps, double cs, T* __restrict__ tiles) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_entries) return;
  double s = 0.0;
  for (int64_t c = ptr[e]; c < ptr[e + 1]; ++c) {
    int32_t k = contrib[c];
    s += eps[k / 36] * Te[k] + cs * Se[k];
  }
  tiles[dest[e]] = (T)s;
}

// Global CSR values: the mass T (with eps) and curl-curl S (with 1/mu)
// interleaved per nonzero; A = T + beta dt^2 S and B1 = 2A - dt^2 S are
// formed inside the products.
__global__ void k_pull_csr(int64_t nnz, const int64_t* __restrict__ ptr, const int32_t* __restrict__ contrib,
                           const double* __restrict__ Te, const double* __restrict__ Se,
                           const double* __restrict__ eps, double2* __restrict__ vals) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  double t = 0.0, s = 0.0;
  for (int64_t c = ptr[e]; c < ptr[e + 1]; ++c) {
    int32_t k = contrib[c];
    t += eps[k / 36] * Te[k];
    s += Se[k];
  }
  vals[e] = make_double2(t, s);
}

// Lumped preconditioner of the interface CG in multiplier space:
// K_lam = sum_s D B_s A_GG^(s) B_s^T D with D = 1/2 (each multiplier joins two
// subdomain copies).  Entry (l, l') sums, over the tets of every subdomain s
// holding both interface edges, 1/4 sign_s(l) sign_s(l') A_e[a][b] with
// A_e = eps T_e + beta dt^2 S_e; contrib = (t*36 + a*6 + b) << 1 | negative.
__global__ void k_pull_lam(int64_t nnz, const int64_t* __restrict__ ptr, const int32_t* __restrict__ contrib,
                           const double* __restrict__ Te, const double* __restrict__ Se,
                           const double* __restrict__ eps, double bdt2, double* __restrict__ vals) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  double v = 0.0;
  for (int64_t c = ptr[e]; c < ptr[e + 1]; ++c) {
    const int32_t code = contrib[c];
    const int32_t k = code >> 1;
    const double a = 0.25 * (eps[k / 36] * Te[k] + bdt2 * Se[k]);
    v += (code & 1) ? -a : a;
  }
  vals[e] = v;
}

// Unit diagonal on padding rows of every tile store (rows that carry no
// unknown), so padded blocks factor to the identity.
template <class T>
__global__ void k_pad_diag(int64_t n, const int64_t* __restrict__ pos, T* __restrict__ tiles) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) tiles[pos[i]] = (T)1;
}

// --------------------------------------------------------------------------
// K2: right-looking tiled partial Cholesky.  For panel k of every subdomain
// with k < kr: (1) factor the diagonal tile and replace it by the inverse of
// its Cholesky factor; (2) panel tiles (i, k) <- A_ik Dinv_k^T for i > k
// (interface and corner rows alike, so corner rows become L_cr);
// (3) trailing tiles (i, j), k < j <= i, -= L_ik L_jk^T (corner block
// becomes K_s = A_cc - L_cr L_cr^T).  Arithmetic in the storage type T
// except the diagonal tile, which is factored and inverted in FP64.
// --------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) k_potrf(int k, int s0, T* __restrict__ tiles,
                                               const SubDev* __restrict__ subs, int* __restrict__ err,
                                               uint8_t* __restrict__ nzl, uint8_t* __restrict__ nzi) {
  const SubDev q = subs[s0 + blockIdx.x];
  if (k >= q.kI + q.kG) return;
  if (threadIdx.x == 0) nzl[tile_index(q, k, k)] = nzi[tile_index(q, k, k)] = 1;
  __shared__ double a[kNB][kNB + 1];
  __shared__ double x[kNB][kNB + 1];
  __shared__ double piv[kNB];
  T* tp = tiles + tile_index(q, k, k) * kTile;
  const int tid = threadIdx.x;
  // thread (rb, c) = (tid / 32, tid % 32) owns entries (rb + 8 u, c), u < 4,
  // kept in registers; LDS holds what other threads read
  constexpr int U = kTile / 256;
  const int c = tid & 31, rb = tid >> 5;
  double v[U], xv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int r = rb + 8 * u;
    v[u] = (double)tp[r * kNB + c];
    a[r][c] = v[u];
    xv[u] = r == c ? 1.0 : 0.0;
    x[r][c] = xv[u];
  }
  __syncthreads();
  // Right-looking elimination with unscaled columns: step j subtracts
  // a_rj a_cj / d_j from the trailing entries (c > j, r >= c) while column j
  // is only read; the owners of column j + 1 publish it for the next step, so
  // one barrier per column.  d_j = pivot; every thread reads the same pivot
  // and takes the same decision on it.
  int bad = 0;
  for (int j = 0; j < kNB; ++j) {
    double d = a[j][j];
    const double acj = a[c][j];
    double arj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) arj[u] = a[rb + 8 * u][j];
    if (!(d > 0.0) || !isfinite(d)) {
      bad = 1;
      d = 1.0;
    }
    const double f = acj / d;
    if (tid == 0) piv[j] = d;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = rb + 8 * u;
      if (c > j && r >= c) v[u] -= arj[u] * f;
      if (c == j + 1) a[r][c] = v[u];
    }
    __syncthreads();
  }
  // L = unscaled columns / sqrt(d)
  const double sd = sqrt(piv[c]);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int r = rb + 8 * u;
    a[r][c] = r < c ? 0.0 : (r == c ? sd : v[u] / sd);
  }
  __syncthreads();
  // L^-1 by forward substitution on the identity, all columns at once: at
  // step m row m is complete up to its division by L_mm, and the rows below
  // take L_rm X_mc / L_mm; the owners of row m + 1 publish it (again one
  // barrier per step)
  for (int m = 0; m < kNB; ++m) {
    const double g = x[m][c] / a[m][m];
    double arm[U];
#pragma unroll
    for (int u = 0; u < U; ++u) arm[u] = a[rb + 8 * u][m];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = rb + 8 * u;
      if (r > m && c <= m) xv[u] -= arm[u] * g;
      if (r == m + 1) x[r][c] = xv[u];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int r = rb + 8 * u;
    tp[r * kNB + c] = (T)(c <= r ? xv[u] / a[r][r] : 0.0);
  }
  if (tid == 0 && bad) atomicMin(err, s0 + (int)blockIdx.x);
}

template <class T>
__global__ void __launch_bounds__(256) k_trsm(int k, int s0, T* __restrict__ tiles,
                                              const SubDev* __restrict__ subs, uint8_t* __restrict__ nzl) {
  const SubDev q = subs[s0 + blockIdx.y];
  const int i = k + 1 + blockIdx.x;
  if (k >= q.kI + q.kG || i >= q.K) return;
  __shared__ T A[kNB][kNB + 1];
  __shared__ T Dv[kNB][kNB + 1];
  T* ap = tiles + tile_index(q, i, k) * kTile;
  const T* dp = tiles + tile_index(q, k, k) * kTile;
  const int tid = threadIdx.x;
  for (int e = tid; e < kTile; e += 256) {
    A[e / kNB][e % kNB] = ap[e];
    Dv[e / kNB][e % kNB] = dp[e];
  }
  __syncthreads();
  // L_ik = A_ik Dinv_k^T on MFMA: wave w computes block (w/2, w%2)
  const int w = tid >> 6, l = tid & 63, mb = w >> 1, nb = w & 1;
  typename Mfma<T>::acc_t acc = {0, 0, 0, 0};
  tile_mma<T, true>(A, Dv, mb, nb, l, acc);
#pragma unroll
  for (int v = 0; v < 4; ++v) ap[(mb * 16 + Mfma<T>::row(l, v)) * kNB + nb * 16 + (l & 15)] = acc[v];
  // nonzero flag of L_ik (a zero tile takes no part in later products)
  const int nz = __syncthreads_or(acc[0] != (T)0 || acc[1] != (T)0 || acc[2] != (T)0 || acc[3] != (T)0);
  if (tid == 0) nzl[tile_index(q, i, k)] = (uint8_t)(nz != 0);
}

// Tile rows of one factor column held by the trailing-update kernel's list.
constexpr int kColList = 8192;

// Trailing update of step k over the nonzero tiles of column k only: every
// workgroup of a subdomain compacts the rows i > k with L_ik != 0 into an LDS
// list, then takes the pairs (a >= b) of that list strided by the grid's x
// size: C_ij -= L_ik L_jk^T.  (A grid over all pairs would dispatch one
// workgroup per trailing tile per step, nearly all of them on zero tiles of
// the nested-dissection order.)  Requires K - k - 1 <= kColList.
template <class T>
__global__ void __launch_bounds__(256) k_syrk(int k, int s0, T* __restrict__ tiles,
                                              const SubDev* __restrict__ subs, const uint8_t* __restrict__ nzl) {
  const SubDev q = subs[s0 + blockIdx.y];
  if (k >= q.kI + q.kG) return;
  const int Tn = q.K - k - 1;
  __shared__ uint16_t list[kColList];
  __shared__ int wcnt[4];
  __shared__ T A[kNB][kNB + 1];
  __shared__ T B[kNB][kNB + 1];
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, mb = w >> 1, nb = w & 1;
  int nn = 0;
  for (int b0 = 0; b0 < Tn; b0 += 256) {
    const int ii = b0 + tid;
    const bool nz = ii < Tn && nzl[tile_index(q, k + 1 + ii, k)];
    const unsigned long long bal = __ballot(nz);
    if (l == 0) wcnt[w] = __popcll(bal);
    __syncthreads();
    int off = nn;
    for (int x = 0; x < w; ++x) off += wcnt[x];
    if (nz) list[off + __popcll(bal & ((1ull << l) - 1ull))] = (uint16_t)ii;
    nn += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    __syncthreads();
  }
  const int64_t npair = (int64_t)nn * (nn + 1) / 2;
  for (int64_t p = blockIdx.x; p < npair; p += gridDim.x) {
    int a = (int)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while ((int64_t)(a + 1) * (a + 2) / 2 <= p) ++a;
    while ((int64_t)a * (a + 1) / 2 > p) --a;
    const int bb = (int)(p - (int64_t)a * (a + 1) / 2);
    const int i = k + 1 + list[a], j = k + 1 + list[bb];
    const T* ap = tiles + tile_index(q, i, k) * kTile;
    const T* bp = tiles + tile_index(q, j, k) * kTile;
    T* cp = tiles + tile_index(q, i, j) * kTile;
    __syncthreads();
    for (int e = tid; e < kTile; e += 256) {
      A[e / kNB][e % kNB] = ap[e];
      B[e / kNB][e % kNB] = bp[e];
    }
    __syncthreads();
    // C_ij -= L_ik L_jk^T on MFMA: wave w computes block (w/2, w%2)
    typename Mfma<T>::acc_t acc = {0, 0, 0, 0};
    tile_mma<T, true>(A, B, mb, nb, l, acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) cp[(mb * 16 + Mfma<T>::row(l, v)) * kNB + nb * 16 + (l & 15)] -= acc[v];
  }
}

// --------------------------------------------------------------------------
// Inversion of the diagonal blocks of the r-block Cholesky factor, one block
// row at a time: Linv_ij = -Dinv_i sum_{m=j}^{i-1} L_im Linv_mj (rows < i
// already inverted, row i still holds L), written to a scratch row, then
// copied back.  Only the I x I block (L_II^-1) and the Gamma x Gamma block
// (L_GG^-1) are inverted; the coupling L_GI stays as the factor left it, so
// that L_rr^-1 w = [L_II^-1 w_I ; L_GG^-1 (w_G - L_GI L_II^-1 w_I)] is applied
// as three products (L_GI has far fewer nonzero tiles than the Gamma x I
// block of L_rr^-1, which is dense).  A block with kG = 0 (the coarse block)
// is inverted whole.
// --------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) k_trtri_row(int i, int s0, const T* __restrict__ tiles,
                                                   const SubDev* __restrict__ subs,
                                                   const int64_t* __restrict__ scratch_off,
                                                   T* __restrict__ scratch, const uint8_t* __restrict__ nzl,
                                                   uint8_t* __restrict__ nzi) {
  const int sidx = s0 + blockIdx.y;
  const SubDev q = subs[sidx];
  const int j = blockIdx.x;
  const int kr = q.kI + q.kG;
  if (i >= kr || j >= i) return;
  if (i >= q.kI && j < q.kI) return;  // L_GI is kept
  __shared__ T A[kNB][kNB + 1];
  __shared__ T B[kNB][kNB + 1];
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, mb = w >> 1, nb = w & 1;
  typename Mfma<T>::acc_t acc = {0, 0, 0, 0};
  // terms with a zero L_im or Linv_mj are skipped
  extern __shared__ uint16_t list[];
  __shared__ int wcnt[4];
  const int nn = chain_list(
      j, i, [&](int m) { return nzl[tile_index(q, i, m)] && nzi[tile_index(q, m, j)]; }, list, wcnt);
  chain_mma<T, false, false>(
      list, nn,
      [&](int m, const T*& ap, const T*& bp) {
        ap = tiles + tile_index(q, i, m) * kTile;  // L_im
        bp = tiles + tile_index(q, m, j) * kTile;  // Linv_mj
      },
      A, B, acc);
  // multiply by -Dinv_i (MFMA again, the sum staged in LDS)
  __syncthreads();
  const T* dp = tiles + tile_index(q, i, i) * kTile;
  for (int e = tid; e < kTile; e += 256) A[e / kNB][e % kNB] = dp[e];
#pragma unroll
  for (int v = 0; v < 4; ++v) B[mb * 16 + Mfma<T>::row(l, v)][nb * 16 + (l & 15)] = acc[v];
  __syncthreads();
  typename Mfma<T>::acc_t out = {0, 0, 0, 0};
  tile_mma<T, false>(A, B, mb, nb, l, out);
  T* sp = scratch + (scratch_off[sidx] + j) * kTile;
#pragma unroll
  for (int v = 0; v < 4; ++v) sp[(mb * 16 + Mfma<T>::row(l, v)) * kNB + nb * 16 + (l & 15)] = -out[v];
  // Linv_ij's flag (rows below i read it; row i's own terms do not)
  const int nz = __syncthreads_or(out[0] != (T)0 || out[1] != (T)0 || out[2] != (T)0 || out[3] != (T)0);
  if (tid == 0) nzi[tile_index(q, i, j)] = (uint8_t)(nz != 0);
}

template <class T>
__global__ void k_trtri_copy(int i, int s0, T* __restrict__ tiles, const SubDev* __restrict__ subs,
                             const int64_t* __restrict__ scratch_off, const T* __restrict__ scratch) {
  const int sidx = s0 + blockIdx.y;
  const SubDev q = subs[sidx];
  const int j = blockIdx.x;
  if (i >= q.kI + q.kG || j >= i) return;
  if (i >= q.kI && j < q.kI) return;  // L_GI is kept
  T* dst = tiles + tile_index(q, i, j) * kTile;
  const T* src = scratch + (scratch_off[sidx] + j) * kTile;
  for (int e = threadIdx.x; e < kTile; e += blockDim.x) dst[e] = src[e];
}

// Corner coupling premultiplied by the interface inverse factor: in corner
// tile row i = kr + c the Gamma columns become Psi_G(i, j) = sum_{m=j}^{kr-1}
// L_cG(i, m) Linv_GG(m, j), kI <= j < kr, i.e. Psi_G = L_cG L_GG^-1 (with
// t = L_rr^-1 w, L_cG t_G = Psi_G y_G for y_G = w_G - L_GI t_I); the I columns
// keep L_cI.  A block with kG = 0 (the coarse block) has no corner rows.
// Written to scratch, then copied.
template <class T>
__global__ void __launch_bounds__(256) k_psi_row(int c, int s0, const T* __restrict__ tiles,
                                                 const SubDev* __restrict__ subs,
                                                 const int64_t* __restrict__ scratch_off, T* __restrict__ scratch,
                                                 const uint8_t* __restrict__ nzl, const uint8_t* __restrict__ nzi) {
  const int sidx = s0 + blockIdx.y;
  const SubDev q = subs[sidx];
  const int j = blockIdx.x;
  const int kr = q.kI + q.kG;
  if (c >= q.kC || j >= kr || j < q.kI) return;
  const int i = kr + c;
  __shared__ T A[kNB][kNB + 1];
  __shared__ T B[kNB][kNB + 1];
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, mb = w >> 1, nb = w & 1;
  typename Mfma<T>::acc_t acc = {0, 0, 0, 0};
  extern __shared__ uint16_t list[];
  __shared__ int wcnt[4];
  const int nn = chain_list(
      j, kr, [&](int m) { return nzl[tile_index(q, i, m)] && nzi[tile_index(q, m, j)]; }, list, wcnt);
  chain_mma<T, false, false>(
      list, nn,
      [&](int m, const T*& ap, const T*& bp) {
        ap = tiles + tile_index(q, i, m) * kTile;  // L_cr(i, m)
        bp = tiles + tile_index(q, m, j) * kTile;  // Linv(m, j)
      },
      A, B, acc);
  T* sp = scratch + (scratch_off[sidx] + j) * kTile;
#pragma unroll
  for (int v = 0; v < 4; ++v) sp[(mb * 16 + Mfma<T>::row(l, v)) * kNB + nb * 16 + (l & 15)] = acc[v];
}

template <class T>
__global__ void k_psi_copy(int c, int s0, T* __restrict__ tiles, const SubDev* __restrict__ subs,
                           const int64_t* __restrict__ scratch_off, const T* __restrict__ scratch) {
  const int sidx = s0 + blockIdx.y;
  const SubDev q = subs[sidx];
  const int j = blockIdx.x;
  const int kr = q.kI + q.kG;
  if (c >= q.kC || j >= kr || j < q.kI) return;
  T* dst = tiles + tile_index(q, kr + c, j) * kTile;
  const T* src = scratch + (scratch_off[sidx] + j) * kTile;
  for (int e = threadIdx.x; e < kTile; e += blockDim.x) dst[e] = src[e];
}

// Coarse corner matrix K_cc = sum_s B_c^T K_s B_c by pull (fixed order).
template <class T>
__global__ void k_pull_coarse(int64_t n, const int64_t* __restrict__ ptr, const int64_t* __restrict__ src,
                              const int64_t* __restrict__ dest, T* __restrict__ tiles) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double s = 0.0;
  for (int64_t c = ptr[e]; c < ptr[e + 1]; ++c) s += (double)tiles[src[c]];
  tiles[dest[e]] = (T)s;
}

// --------------------------------------------------------------------------
// Batched tile products for the solves (the substitutions, applied through
// the stored inverse factors).
//
// Solve-phase tile layout ("operand order"): lane l = 16g + i of a wave
// holds the 8 values (row mb*16+i, columns 8g..8g+7) of row block mb, laid
// out so that each 16-byte load instruction of the wave reads one contiguous
// kilobyte (swz / load_chunk8): a whole tile is one fully coalesced sweep.  The store used for products with the tile
// itself (NOTRANS) holds each tile in this order; a second store holds the
// transposed tiles in the same order (TRANS).  Within one 16x16x4 MFMA the
// reduction index of lane group g at step ks is column 8g + ks, so the
// operand of every lane is a register of its contiguous chunk.
//
// One work item = one wave = (subdomain, output block o, tile range
// [lo, hi)); with a tile list (mlist != null, used for the sparse coarse
// inverse factor) the range indexes mlist and m = mlist[k].  NOTRANS tiles
// are (o, m), TRANS tiles (m, o), input block m:
//     NOTRANS: acc = sum_m tile(o,m) in_m      TRANS: acc = sum_m tile(m,o)^T in_m
// slot < 0: out_o = (add ? add_o : 0) + alpha acc; output blocks in the
// corner rows (o >= kr) use add_c / alpha_c instead.  Long ranges are split
// into chunks: each chunk writes partial[slot] and k_mv_reduce sums the
// slots of each output block in slot order (deterministic).  (A last-wave
// reduction inside this kernel needs device-scope release/acquire fences,
// which write back / invalidate the per-XCD L2 and cost far more than the
// extra launch.)
// Modes: nrhs <= NV uses vector FMAs (lanes of a column group reduced with
// cross-lane shuffles); nrhs in 9..32 uses MFMA 16x16x4 in 16-wide RHS
// blocks (NB16 of them).
// --------------------------------------------------------------------------
struct MvItem {
  int32_t s, o, lo, hi;  // subdomain, output block, tile range [lo, hi)
  int32_t slot;          // -1: write the output block; else partial slot
  int32_t oidx;          // split items: index of the output block's MvOut
  int32_t o2 = -1;       // row-pair lists: second output block (-1: none)
  int32_t slot2 = -1;    // its partial slot (-1: write it directly)
};

// Full-pass tile lists flag the 16 x 16 quarters of a tile that are all
// zero (bit 2 * row half + column half, the layout of the store read), so
// that the lanes of such a quarter read the cached zero tile instead of
// memory.  Single-row lists: entry = m | zero quarters << 25.  Row-pair
// lists: entry = m | zero quarters of (o, m) << 21 | of (o2, m) << 25 |
// (tile (o, m) present) << 29 | (tile (o2, m) present) << 30 (transposed
// pass: tiles (m, o) and (m, o2)).
constexpr int32_t kListMask = (1 << 25) - 1;
constexpr int32_t kPairMask = (1 << 21) - 1;

// --------------------------------------------------------------------------
// V consecutive right-hand sides of one row in single loads / stores (the
// row slice is aligned to 4V bytes for float and to 16 bytes for double:
// rows hold nrhs entries, nrhs a multiple of V, and buffers are 256-byte
// aligned).  The vector forms of the multiplier-space kernels below give
// each lane V right-hand sides, so index loads are shared by nrhs / V lanes
// instead of nrhs and each gather moves 4V or 8V contiguous bytes.
// --------------------------------------------------------------------------
template <class T, int V>
__device__ __forceinline__ void vload(const T* __restrict__ p, T (&o)[V]) {
  static_assert(V == 2 || V == 4, "vector width");
  if constexpr (sizeof(T) == 4 && V == 4) {
    const float4 t = *reinterpret_cast<const float4*>(p);
    o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
  } else if constexpr (sizeof(T) == 4) {
    const float2 t = *reinterpret_cast<const float2*>(p);
    o[0] = t.x; o[1] = t.y;
  } else {
#pragma unroll
    for (int h = 0; h < V / 2; ++h) {
      const double2 t = reinterpret_cast<const double2*>(p)[h];
      o[2 * h] = t.x; o[2 * h + 1] = t.y;
    }
  }
}

template <class T, int V>
__device__ __forceinline__ void vstore(T* __restrict__ p, const T (&o)[V]) {
  static_assert(V == 2 || V == 4, "vector width");
  if constexpr (sizeof(T) == 4 && V == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(o[0], o[1], o[2], o[3]);
  } else if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<float2*>(p) = make_float2(o[0], o[1]);
  } else {
#pragma unroll
    for (int h = 0; h < V / 2; ++h) reinterpret_cast<double2*>(p)[h] = make_double2(o[2 * h], o[2 * h + 1]);
  }
}

// block partials of per-RHS sums held V to a lane: lane (l, q), l < lpr,
// q < G = nrhs / V, holds right-hand sides q V .. q V + V - 1; summed over l
// in lane order.  Ends with a barrier (callable twice in a row).
template <int V>
__device__ __forceinline__ void block_rhs_sum_v(const double (&s)[V], int nrhs, int lpr,
                                                double* __restrict__ partial) {
  __shared__ double red[256 * V];
  const int tid = threadIdx.x, G = nrhs / V;
#pragma unroll
  for (int v = 0; v < V; ++v) red[tid * V + v] = s[v];
  __syncthreads();
  if (tid < nrhs) {
    const int q = tid / V, v = tid % V;
    double t = 0.0;
    for (int l = 0; l < lpr; ++l) t += red[(l * G + q) * V + v];
    partial[blockIdx.x * kMaxRhs + tid] = t;
  }
  __syncthreads();
}

struct MvOut {
  int32_t s, o, slot0, nslot;
};

// operand-order position of logical element (r, c) of a tile: row block
// mb = r/16, lane l = 16*(c/8) + r%16, value k = c%8 of that lane, stored
// as vector q = k/V, component k%V, V = 16/sizeof(T) (see load_chunk8)
template <class T>
__device__ __forceinline__ int swz(int r, int c) {
  constexpr int V = 16 / sizeof(T);
  const int l = 16 * (c >> 3) + (r & 15), k = c & 7;
  return (r >> 4) * 512 + (k / V) * 64 * V + l * V + (k % V);
}


typedef float f32x4v __attribute__((ext_vector_type(4)));
typedef double f64x2v __attribute__((ext_vector_type(2)));

// 8 values of lane l from one row block (512 elements) in operand order:
// the q-th 16-byte vector of every lane sits at q*64*V + l*V (V = 16/sizeof(T)),
// so each load instruction of the wave reads one contiguous kilobyte.
// (Non-temporal hints on these loads were measured slower.)
template <class T>
__device__ __forceinline__ void load_chunk8(const T* __restrict__ blk, int l, T* v) {
  if constexpr (sizeof(T) == 4) {
    const f32x4v* q = reinterpret_cast<const f32x4v*>(blk);
    f32x4v a = q[l], b = q[64 + l];
    v[0] = a[0]; v[1] = a[1]; v[2] = a[2]; v[3] = a[3];
    v[4] = b[0]; v[5] = b[1]; v[6] = b[2]; v[7] = b[3];
  } else {
    const f64x2v* q = reinterpret_cast<const f64x2v*>(blk);
    f64x2v a = q[l], b = q[64 + l], c = q[128 + l], d = q[192 + l];
    v[0] = a[0]; v[1] = a[1]; v[2] = b[0]; v[3] = b[1];
    v[4] = c[0]; v[5] = c[1]; v[6] = d[0]; v[7] = d[1];
  }
}

// NV > 0: vector path for nrhs <= NV; NV == 0: MFMA path with NB16 RHS blocks.
// CLS only names the product class in kernel traces (0 interface blocks of
// the inverse factors, 1 full r-blocks, 3 coarse, 4 corner rows).
template <class T, int NV, int NB16, int CLS, int LD>
__global__ void __launch_bounds__(256) k_tile_mv(int64_t n_items, const MvItem* __restrict__ items,
                                                 const SubDev* __restrict__ subs, const T* __restrict__ tiles,
                                                 const T* __restrict__ in, T* __restrict__ out,
                                                 const T* __restrict__ add, T alpha, const T* __restrict__ add_c,
                                                 T alpha_c, int nrhs_rt, int trans, T* __restrict__ partial,
                                                 const int32_t* __restrict__ mlist, const int* __restrict__ skip,
                                                 const T* __restrict__ zero) {
  if (skip && *skip) return;
  // LD > 0: the RHS count is LD (= 16 NB16), a compile-time row stride
  const int nrhs = LD > 0 ? LD : nrhs_rt;
  // Work groups of 4 items (one per wave); workgroup b takes groups b,
  // b + gridDim.x, ...: one pass over the list with as many workgroups as
  // groups, or a persistent grid (a multiple of 8, so that every group a
  // workgroup takes was placed on that workgroup's XCD).  No workgroup
  // barriers: the waves of a workgroup are independent.
  const int64_t ngroups = (n_items + 3) / 4;
  for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int64_t wi = grp * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
    if (wi >= n_items) continue;
    const MvItem w = items[wi];
    if (w.s < 0) continue;  // padding item
    const SubDev q = subs[w.s];
    const int l = threadIdx.x & 63;
    const int g = l >> 4, i = l & 15;
    const T* xbase = in + q.row_off * nrhs;
    constexpr bool MF = NV == 0;
    constexpr int NA = MF ? 2 * NB16 : 2 * NV;
    // accumulators: vector path acc[mb*NV + r]; MFMA path acc[mb*NB16 + nb]
    typename Mfma<T>::acc_t macc[MF ? 2 * NB16 : 1];
    T vacc[MF ? 1 : NA];
    if constexpr (MF) {
#pragma unroll
      for (int a = 0; a < 2 * NB16; ++a) macc[a] = typename Mfma<T>::acc_t{0, 0, 0, 0};
    } else {
#pragma unroll
      for (int a = 0; a < NA; ++a) vacc[a] = 0;
    }
    // factor values of the current / next tile, and (prefetched together with
    // them) the input values the lane needs: MFMA path bv[nb][ks] = x[8g+ks][nb*16+i],
    // vector path (NV <= 2) x[8g+ks][r]; wider vector paths load x inline
    constexpr bool PX = MF || NV <= 2;
    constexpr int NX = PX ? 8 * (MF ? NB16 : NV) : 1;
    T cur[16], nxt[16], xc[NX], xn[NX];
    auto tile_ptr = [&](int m) -> const T* {
      const int ti = trans ? m : w.o, tj = trans ? w.o : m;
      return tiles + tile_index(q, ti, tj) * kTile;
    };
    // Loads are unconditional (clamped to an in-bounds column, then zeroed
    // by a select): a masked load compiles to a branch whose other arm waits
    // for every load in flight, prefetches included.
    auto load_x = [&](int m, T* xv) {
      const T* xb = xbase + (int64_t)m * kNB * nrhs;
      if constexpr (MF) {
#pragma unroll
        for (int nb = 0; nb < NB16; ++nb) {
          const int col = nb * 16 + i;
          const int cc = col < nrhs ? col : nrhs - 1;
#pragma unroll
          for (int ks = 0; ks < 8; ++ks) {
            const T v = xb[(8 * g + ks) * nrhs + cc];
            xv[nb * 8 + ks] = col < nrhs ? v : (T)0;
          }
        }
      } else if constexpr (PX) {
#pragma unroll
        for (int ks = 0; ks < 8; ++ks)
#pragma unroll
          for (int r = 0; r < NV; ++r) {
            const T v = xb[(8 * g + ks) * nrhs + (r < nrhs ? r : nrhs - 1)];
            xv[ks * NV + r] = r < nrhs ? v : (T)0;
          }
      }
    };
    auto ent = [&](int k) -> int32_t { return mlist ? mlist[k] : k; };
    // a lane reads the zero tile for the quarters flagged all-zero (lane
    // group g holds columns 8g..8g+7: column half g / 2)
    auto load_tile = [&](int32_t e, T* c) {
      const T* tp = tile_ptr(e & kListMask);
      const int zq = (e >> 25) & 15, ch = g >> 1;
      load_chunk8(((zq >> ch) & 1) ? zero : tp, l, c);
      load_chunk8((((zq >> (2 + ch)) & 1) ? zero : tp) + 512, l, c + 8);
    };
    if constexpr (MF) {
      // two tiles (and their input blocks) in flight: a ring of three
      // buffers over the item's tiles, the loop unrolled by three so that
      // each buffer stays in fixed registers (no copies between iterations)
      T rb[3][16], rx[3][NX];
      auto ld = [&](int k, int u) {
        const int32_t e = ent(k);
        load_tile(e, rb[u]);
        load_x(e & kListMask, rx[u]);
      };
      auto mm = [&](int u) {
#pragma unroll
        for (int nb = 0; nb < NB16; ++nb)
#pragma unroll
          for (int ks = 0; ks < 8; ++ks) {
            macc[nb] = Mfma<T>::op(rb[u][ks], rx[u][nb * 8 + ks], macc[nb]);
            macc[NB16 + nb] = Mfma<T>::op(rb[u][8 + ks], rx[u][nb * 8 + ks], macc[NB16 + nb]);
          }
      };
      if (w.lo < w.hi) ld(w.lo, 0);
      if (w.lo + 1 < w.hi) ld(w.lo + 1, 1);
      for (int k = w.lo; k < w.hi; k += 3) {
        if (k + 2 < w.hi) ld(k + 2, 2);
        mm(0);
        if (k + 3 < w.hi) ld(k + 3, 0);
        if (k + 1 < w.hi) mm(1);
        if (k + 4 < w.hi) ld(k + 4, 1);
        if (k + 2 < w.hi) mm(2);
      }
    }
    if (!MF && w.lo < w.hi) {
      const int32_t e0 = ent(w.lo);
      load_tile(e0, cur);
      load_x(e0 & kListMask, xc);
    }
    // vector path: one tile in flight
    for (int k = w.lo; k < (MF ? w.lo : w.hi); ++k) {
      const int m = ent(k) & kListMask;
      if (k + 1 < w.hi) {
        const int32_t e1 = ent(k + 1);
        load_tile(e1, nxt);
        load_x(e1 & kListMask, xn);
      }
      if constexpr (PX) {
#pragma unroll
        for (int ks = 0; ks < 8; ++ks)
#pragma unroll
          for (int r = 0; r < NV; ++r) {
            vacc[r] += cur[ks] * xc[ks * NV + r];
            vacc[NV + r] += cur[8 + ks] * xc[ks * NV + r];
          }
      } else {
        const T* xb = xbase + (int64_t)m * kNB * nrhs;
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
          const T* xr = xb + (8 * g + ks) * nrhs;
#pragma unroll
          for (int r = 0; r < NV; ++r) {
            if (r < nrhs) {
              const T xv = xr[r];
              vacc[r] += cur[ks] * xv;
              vacc[NV + r] += cur[8 + ks] * xv;
            }
          }
        }
      }
      if (k + 1 < w.hi) {
#pragma unroll
        for (int u = 0; u < 16; ++u) cur[u] = nxt[u];
        if constexpr (PX) {
#pragma unroll
          for (int u = 0; u < NX; ++u) xc[u] = xn[u];
        }
      }
    }
    // ---- epilogue ------------------------------------------------------------
    T* dst;
    const T* adp = nullptr;
    T scale;
    if (w.slot < 0) {
      // corner output rows (o >= kr) take their own alpha / add
      const bool crow = w.o >= q.kI + q.kG;
      const T* ad = crow ? add_c : add;
      dst = out + (q.row_off + (int64_t)w.o * kNB) * nrhs;
      if (ad) adp = ad + (q.row_off + (int64_t)w.o * kNB) * nrhs;
      scale = crow ? alpha_c : alpha;
    } else {
      dst = partial + (int64_t)w.slot * kNB * nrhs;
      scale = (T)1;
    }
    if constexpr (MF) {
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB16; ++nb) {
          const int col = nb * 16 + i;
          if (col < nrhs) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = mb * 16 + Mfma<T>::row(l, v);
              const int64_t o = (int64_t)row * nrhs + col;
              T val = scale * macc[mb * NB16 + nb][v];
              if (adp) val += adp[o];
              dst[o] = val;
            }
          }
        }
    } else {
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        T v = vacc[a];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        vacc[a] = v;
      }
      // lane group g writes right-hand sides r with r % 4 == g
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int r = 0; r < NV; ++r) {
          if (r < nrhs && (r & 3) == g) {
            const int64_t o = (int64_t)(mb * 16 + i) * nrhs + r;
            T val = scale * vacc[mb * NV + r];
            if (adp) val += adp[o];
            dst[o] = val;
          }
        }
    }
  }  // groups
}

// Row-pair form of k_tile_mv for the full passes (MFMA path, 9..32 RHS):
// one wave computes the output blocks o and o2 of one subdomain over the
// union of their tile lists, so each input block is loaded once for both
// rows (the input loads cost about as much as a tile's own once they are
// not shared).  An entry's absent tile is read from `zero`, one zero tile
// (cached after its first use).  Split items write partial slots w.slot
// (block o) and w.slot2 (block o2), as k_tile_mv does.
template <class T, int NB16, int CLS, int LD>
__global__ void __launch_bounds__(256) k_tile_mv2(int64_t n_items, const MvItem* __restrict__ items,
                                                  const SubDev* __restrict__ subs, const T* __restrict__ tiles,
                                                  const T* __restrict__ in, T* __restrict__ out,
                                                  const T* __restrict__ add, T alpha, const T* __restrict__ add_c,
                                                  T alpha_c, int nrhs_rt, int trans, T* __restrict__ partial,
                                                  const int32_t* __restrict__ mlist, const int* __restrict__ skip,
                                                  const T* __restrict__ zero) {
  if (skip && *skip) return;
  // LD > 0: the RHS count is LD (= 16 NB16), a compile-time row stride
  const int nrhs = LD > 0 ? LD : nrhs_rt;
  const int64_t ngroups = (n_items + 3) / 4;
  for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int64_t wi = grp * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wave
    if (wi >= n_items) continue;
    const MvItem w = items[wi];
    if (w.s < 0) continue;  // padding item
    const SubDev q = subs[w.s];
    const int l = threadIdx.x & 63;
    const int g = l >> 4, i = l & 15;
    const T* xbase = in + q.row_off * nrhs;
    const bool two = w.o2 >= 0;
    using acc_t = typename Mfma<T>::acc_t;
    acc_t acc[2][2 * NB16];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int a = 0; a < 2 * NB16; ++a) acc[p][a] = acc_t{0, 0, 0, 0};
    // tiles of the current / next entry for both rows, and the input block
    T cur[2][16], nxt[2][16], xc[8 * NB16], xn[8 * NB16];
    auto tptr = [&](int o, int m, bool present) -> const T* {
      if (!present) return zero;
      const int ti = trans ? m : o, tj = trans ? o : m;
      return tiles + tile_index(q, ti, tj) * kTile;
    };
    auto load_x = [&](int m, T* xv) {
      const T* xb = xbase + (int64_t)m * kNB * nrhs;
#pragma unroll
      for (int nb = 0; nb < NB16; ++nb) {
        const int col = nb * 16 + i;
        const int cc = col < nrhs ? col : nrhs - 1;
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
          const T v = xb[(8 * g + ks) * nrhs + cc];
          xv[nb * 8 + ks] = col < nrhs ? v : (T)0;
        }
      }
    };
    const int ch = g >> 1;  // column half of this lane's values
    auto load_entry = [&](int k, T (&t)[2][16], T* xv) {
      const int32_t e = mlist[k];
      const int m = e & kPairMask;
      const int za = (e >> 21) & 15, zb = (e >> 25) & 15;
      const T* pa = tptr(w.o, m, (e >> 29) & 1);
      const T* pb = tptr(two ? w.o2 : w.o, m, two && ((e >> 30) & 1));
      load_chunk8(((za >> ch) & 1) ? zero : pa, l, t[0]);
      load_chunk8((((za >> (2 + ch)) & 1) ? zero : pa) + 512, l, t[0] + 8);
      load_chunk8(((zb >> ch) & 1) ? zero : pb, l, t[1]);
      load_chunk8((((zb >> (2 + ch)) & 1) ? zero : pb) + 512, l, t[1] + 8);
      load_x(m, xv);
    };
    if (w.lo < w.hi) load_entry(w.lo, cur, xc);
    for (int k = w.lo; k < w.hi; ++k) {
      if (k + 1 < w.hi) load_entry(k + 1, nxt, xn);
#pragma unroll
      for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int nb = 0; nb < NB16; ++nb)
#pragma unroll
          for (int ks = 0; ks < 8; ++ks) {
            acc[p][nb] = Mfma<T>::op(cur[p][ks], xc[nb * 8 + ks], acc[p][nb]);
            acc[p][NB16 + nb] = Mfma<T>::op(cur[p][8 + ks], xc[nb * 8 + ks], acc[p][NB16 + nb]);
          }
      if (k + 1 < w.hi) {
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int u = 0; u < 16; ++u) cur[p][u] = nxt[p][u];
#pragma unroll
        for (int u = 0; u < 8 * NB16; ++u) xc[u] = xn[u];
      }
    }
    // ---- epilogue: both output blocks ------------------------------------
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      if (p == 1 && !two) break;
      const int o = p ? w.o2 : w.o;
      const int slot = p ? w.slot2 : w.slot;
      T* dst;
      const T* adp = nullptr;
      T scale;
      if (slot < 0) {
        const bool crow = o >= q.kI + q.kG;
        const T* ad = crow ? add_c : add;
        dst = out + (q.row_off + (int64_t)o * kNB) * nrhs;
        if (ad) adp = ad + (q.row_off + (int64_t)o * kNB) * nrhs;
        scale = crow ? alpha_c : alpha;
      } else {
        dst = partial + (int64_t)slot * kNB * nrhs;
        scale = (T)1;
      }
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB16; ++nb) {
          const int col = nb * 16 + i;
          if (col < nrhs) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = mb * 16 + Mfma<T>::row(l, v);
              const int64_t oo = (int64_t)row * nrhs + col;
              T val = scale * acc[p][mb * NB16 + nb][v];
              if (adp) val += adp[oo];
              dst[oo] = val;
            }
          }
        }
    }
  }  // groups
}

// Row-octet form for the full passes (MFMA path, 9..32 RHS): a workgroup
// item covers up to 8 consecutive output rows o .. o + w.o2 - 1 of one
// subdomain over the union of their tile lists; each entry's input block is
// staged once in LDS (transposed: a lane's 8 reduction values are
// contiguous) and used by all four waves, wave v computing rows o + 2v and
// o + 2v + 1.  Entry = m | (tile of row o + j present) << (23 + j); an absent
// tile reads `zero`.  Double-buffered LDS, one workgroup barrier per entry;
// outputs are written directly (octet items are not split).
constexpr int32_t kOctMask = (1 << 23) - 1;
template <class T, int NB16, int CLS, int LD>
__global__ void __launch_bounds__(256) k_tile_mv8(int64_t n_items, const MvItem* __restrict__ items,
                                                  const SubDev* __restrict__ subs, const T* __restrict__ tiles,
                                                  const T* __restrict__ in, T* __restrict__ out,
                                                  const T* __restrict__ add, T alpha, const T* __restrict__ add_c,
                                                  T alpha_c, int nrhs_rt, int trans, const int32_t* __restrict__ mlist,
                                                  const int* __restrict__ skip, const T* __restrict__ zero) {
  if (skip && *skip) return;
  // LD > 0: the RHS count is LD (= 16 NB16), a compile-time row stride
  const int nrhs = LD > 0 ? LD : nrhs_rt;
  constexpr int LP = kNB + 4;            // LDS pitch of one RHS column (16-byte multiple)
  constexpr int XPER = (kNB * 16 * NB16 + 255) / 256;
  __shared__ __align__(16) T xs[2][16 * NB16][LP];
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63, g = l >> 4, i = l & 15;
  const int t = threadIdx.x;
  using acc_t = typename Mfma<T>::acc_t;
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x) {
    const MvItem w = items[it];
    if (w.s < 0) continue;  // uniform over the workgroup
    const SubDev q = subs[w.s];
    const T* xbase = in + q.row_off * nrhs;
    const int ra = 2 * wv, rb = 2 * wv + 1;  // this wave's rows within the octet
    acc_t acc[2][2 * NB16];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int a = 0; a < 2 * NB16; ++a) acc[p][a] = acc_t{0, 0, 0, 0};
    T cur[2][16], nxt[2][16], xr[XPER];
    auto tptr = [&](int j, int m, int32_t e) -> const T* {
      if (j >= w.o2 || !((e >> (23 + j)) & 1)) return zero;
      const int o = w.o + j;
      const int ti = trans ? m : o, tj = trans ? o : m;
      return tiles + tile_index(q, ti, tj) * kTile;
    };
    auto load_tiles = [&](int32_t e, T (&c)[2][16]) {
      const int m = e & kOctMask;
      const T* pa = tptr(ra, m, e);
      const T* pb = tptr(rb, m, e);
      load_chunk8(pa, l, c[0]);
      load_chunk8(pa + 512, l, c[0] + 8);
      load_chunk8(pb, l, c[1]);
      load_chunk8(pb + 512, l, c[1] + 8);
    };
    // input block m ([32 rows][nrhs], row-major) -> registers -> LDS [col][row]
    auto stage_load = [&](int32_t e) {
      const T* xb = xbase + (int64_t)(e & kOctMask) * kNB * nrhs;
#pragma unroll
      for (int j = 0; j < XPER; ++j) {
        const int idx = t + 256 * j;
        const int cl = idx < kNB * nrhs ? idx : 0;
        const T v = xb[cl];
        xr[j] = idx < kNB * nrhs ? v : (T)0;
      }
    };
    auto stage_store = [&](int buf) {
#pragma unroll
      for (int j = 0; j < XPER; ++j) {
        const int idx = t + 256 * j;
        if (idx < kNB * nrhs) xs[buf][idx % nrhs][idx / nrhs] = xr[j];
      }
    };
    if (w.lo < w.hi) {  // (an empty octet writes add + 0: uniform over the workgroup)
      int32_t e = mlist[w.lo];
      stage_load(e);
      load_tiles(e, cur);
      stage_store(0);
      __syncthreads();
      for (int k = w.lo; k < w.hi; ++k) {
        const int buf = (k - w.lo) & 1;
        const bool more = k + 1 < w.hi;
        if (more) {
          e = mlist[k + 1];
          stage_load(e);
          load_tiles(e, nxt);
        }
        T xv[8 * NB16];
#pragma unroll
        for (int nb = 0; nb < NB16; ++nb) {
          const int col = nb * 16 + i;
#pragma unroll
          for (int ks = 0; ks < 8; ++ks) xv[nb * 8 + ks] = col < nrhs ? xs[buf][col][8 * g + ks] : (T)0;
        }
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
          for (int nb = 0; nb < NB16; ++nb)
#pragma unroll
            for (int ks = 0; ks < 8; ++ks) {
              acc[p][nb] = Mfma<T>::op(cur[p][ks], xv[nb * 8 + ks], acc[p][nb]);
              acc[p][NB16 + nb] = Mfma<T>::op(cur[p][8 + ks], xv[nb * 8 + ks], acc[p][NB16 + nb]);
            }
        if (more) stage_store(buf ^ 1);
        __syncthreads();
        if (more) {
#pragma unroll
          for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int u = 0; u < 16; ++u) cur[p][u] = nxt[p][u];
        }
      }
    }
    // ---- epilogue: this wave's two rows ----------------------------------
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int j = p ? rb : ra;
      if (j >= w.o2) continue;
      const int o = w.o + j;
      const bool crow = o >= q.kI + q.kG;
      const T* ad = crow ? add_c : add;
      T* dst = out + (q.row_off + (int64_t)o * kNB) * nrhs;
      const T* adp = ad ? ad + (q.row_off + (int64_t)o * kNB) * nrhs : nullptr;
      const T scale = crow ? alpha_c : alpha;
#pragma unroll
      for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB16; ++nb) {
          const int col = nb * 16 + i;
          if (col < nrhs) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = mb * 16 + Mfma<T>::row(l, v);
              const int64_t oo = (int64_t)row * nrhs + col;
              T val = scale * acc[p][mb * NB16 + nb][v];
              if (adp) val += adp[oo];
              dst[oo] = val;
            }
          }
        }
    }
  }
}

// --------------------------------------------------------------------------
// Symmetric product y = M u with only the lower tiles of M stored (M: the
// interface block of a subdomain's local inverse).  Every tile is read once
// and used twice.  Interface tiles are grouped into panels of PW; one wave
// takes the tiles (o, m), m <= o, of a panel pair (P, Q), P >= Q:
//     row part     y_o += M_om u_m      (o in panel P)
//     column part  y_m += M_om^T u_o    (m in panel Q, m < o)
// accumulated in registers (MFMA 16x16x4, NB16 blocks of 16 RHS; smaller RHS
// counts are zero-padded).  The column part needs the tile with lanes along
// its columns: each wave stages the tile in its own LDS area and reads it back
// transposed (only wave-level ordering is involved).
// Output block b (interface tile index) gets exactly one partial from every
// panel j: slot slot0 + b nP + j holds the row part of pair (P(b), j) for
// j < P(b), the diagonal pair's sum for j = P(b), and the column part of pair
// (j, P(b)) for j > P(b); k_mv_reduce sums them in panel order.
// --------------------------------------------------------------------------
struct SymItem {
  int32_t s, P, Q;  // subdomain, panel pair (P >= Q)
  int32_t slot0;    // first partial slot of the subdomain (kG * nP slots)
};

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

#ifndef SYMV_DEPTH
#define SYMV_DEPTH 2  // FP32 tiles in flight per wave in k_symv
#endif
// FP32 at 16 RHS fits three waves per SIMD without spills (the stream of
// tiles needs the loads of more waves in flight).
template <class T, int NB16, int PW, int LD>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LD == 16 && sizeof(T) == 4 && (SYMV_DEPTH == 1 || PW == 2) ? 3 : 1))) k_symv(int64_t n_items, const SymItem* __restrict__ items,
                                              const SubDev* __restrict__ subs, const int64_t* __restrict__ m_off,
                                              const T* __restrict__ mt, const T* __restrict__ in,
                                              T* __restrict__ partial, int nrhs_rt, const int* __restrict__ skip,
                                              const T* __restrict__ zero) {
  // LD > 0: the RHS count is LD (= 16 NB16), a compile-time row stride
  const int nrhs = LD > 0 ? LD : nrhs_rt;
  if (skip && *skip) return;
  __shared__ T lds[4][kNB][kNB + 1];
  // the wave index is uniform over the wave: item, subdomain record and
  // tile addresses go to scalar registers
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // one item per wave; a grid smaller than the item groups walks them
  // (groups b, b + G, ...: G a multiple of 8 keeps a workgroup on its XCD).
  // No workgroup barriers below: waves are independent.
  for (int64_t wi = (int64_t)blockIdx.x * 4 + wv; wi < n_items; wi += (int64_t)gridDim.x * 4) {
    const SymItem it = items[wi];
    if (it.s < 0) continue;
    const SubDev q = subs[it.s];
    const int l = threadIdx.x & 63, g = l >> 4, i = l & 15;
    const int kG = q.kG;
    const int nP = (kG + PW - 1) / PW;
    const bool diag = it.P == it.Q;
    const int o0 = it.P * PW, m0 = it.Q * PW;
    const T* mb = mt + m_off[it.s] * kTile;
    const T* xg = in + (q.row_off + (int64_t)q.kI * kNB) * nrhs;
    T(*sh)[kNB + 1] = lds[wv];
    using acc_t = typename Mfma<T>::acc_t;
    acc_t racc[PW][2][NB16], cacc[PW][2][NB16];
#pragma unroll
    for (int a = 0; a < PW; ++a)
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int nb = 0; nb < NB16; ++nb) {
          racc[a][h][nb] = acc_t{0, 0, 0, 0};
          cacc[a][h][nb] = acc_t{0, 0, 0, 0};
        }
    auto valid = [&](int t) -> bool {
      const int jr = t / PW, jc = t % PW;
      return o0 + jr < kG && m0 + jc < kG && (!diag || jc <= jr);
    };
    auto tile_of = [&](int t) -> const T* {
      const int o = o0 + t / PW, m = m0 + t % PW;
      return mb + ((int64_t)o * (o + 1) / 2 + m) * kTile;
    };
    // xv[nb*8 + ks] = u[block b][row 8g + ks][rhs nb*16 + i]
    // (unconditional loads from a clamped column, as in k_tile_mv)
    auto load_x = [&](int b, T* xv) {
      const T* xb = xg + (int64_t)b * kNB * nrhs;
#pragma unroll
      for (int nb = 0; nb < NB16; ++nb) {
        const int col = nb * 16 + i;
        const int cc = col < nrhs ? col : nrhs - 1;
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
          const T v = xb[(8 * g + ks) * nrhs + cc];
          xv[nb * 8 + ks] = col < nrhs ? v : (T)0;
        }
      }
    };
    // Static schedule over the PW x PW positions of the pair (all indices
    // compile-time after unrolling, so the ring buffers need no copies): tile
    // t + D and its u_m block are loaded while tile t is used.  A position
    // outside the stored triangle or past the last interface tile reads the
    // zero tile (its u_m block clamped in range), so its products add zero;
    // every load is unconditional.  u_o changes with the row: the next row's
    // block is loaded when the current row starts.
    constexpr int DEPTH = sizeof(T) == 4 ? SYMV_DEPTH : 1;
    constexpr int NT = PW * PW, NBUF = DEPTH + 1;
    T tb[NBUF][16], xb[NBUF][8 * NB16], xo[8 * NB16], xon[8 * NB16];
    auto tile_addr = [&](int t) -> const T* { return valid(t) ? tile_of(t) : zero; };
    auto clampb = [&](int b) { return b < kG ? b : kG - 1; };
    auto prefetch = [&](int t) {
      const T* tp = tile_addr(t);
      load_chunk8(tp, l, tb[t % NBUF]);
      load_chunk8(tp + 512, l, tb[t % NBUF] + 8);
      load_x(clampb(m0 + t % PW), xb[t % NBUF]);
    };
#pragma unroll
    for (int t = 0; t < DEPTH && t < NT; ++t) prefetch(t);
    load_x(o0, xo);
    if (PW > 1) load_x(clampb(o0 + 1), xon);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int jr = t / PW, jc = t % PW;
      if (jc == 0 && jr > 0) {
#pragma unroll
        for (int u = 0; u < 8 * NB16; ++u) xo[u] = xon[u];
        if (jr + 1 < PW) load_x(clampb(o0 + jr + 1), xon);
      }
      if (t + DEPTH < NT) prefetch(t + DEPTH);
      const T* cur = tb[t % NBUF];
      const T* xm = xb[t % NBUF];
#pragma unroll
      for (int nb = 0; nb < NB16; ++nb)
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
          racc[jr][0][nb] = Mfma<T>::op(cur[ks], xm[nb * 8 + ks], racc[jr][0][nb]);
          racc[jr][1][nb] = Mfma<T>::op(cur[8 + ks], xm[nb * 8 + ks], racc[jr][1][nb]);
        }
      // the column part of a diagonal tile would count it twice; above the
      // diagonal of a diagonal pair the tile is zero
      if (!diag || jc < jr) {
        // column part: lane (g, i) needs M(8g + ks, cb*16 + i)
        wave_lds_sync();
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int ks = 0; ks < 8; ++ks) sh[h * 16 + i][8 * g + ks] = cur[h * 8 + ks];
        wave_lds_sync();
        T tt[16];
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
          for (int ks = 0; ks < 8; ++ks) tt[cb * 8 + ks] = sh[8 * g + ks][cb * 16 + i];
#pragma unroll
        for (int nb = 0; nb < NB16; ++nb)
#pragma unroll
          for (int ks = 0; ks < 8; ++ks) {
            cacc[jc][0][nb] = Mfma<T>::op(tt[ks], xo[nb * 8 + ks], cacc[jc][0][nb]);
            cacc[jc][1][nb] = Mfma<T>::op(tt[8 + ks], xo[nb * 8 + ks], cacc[jc][1][nb]);
          }
      }
    }
    // ---- partial blocks ---------------------------------------------------------
    auto write = [&](int b, int j, const acc_t (&a)[2][NB16], const acc_t (&c)[2][NB16], bool both) {
      T* dst = partial + (int64_t)(it.slot0 + b * nP + j) * kNB * nrhs;
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int nb = 0; nb < NB16; ++nb) {
          const int col = nb * 16 + i;
          if (col < nrhs) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = h * 16 + Mfma<T>::row(l, v);
              dst[(int64_t)row * nrhs + col] = both ? a[h][nb][v] + c[h][nb][v] : a[h][nb][v];
            }
          }
        }
    };
#pragma unroll
    for (int j = 0; j < PW; ++j) {
      if (o0 + j < kG) {
        if (diag)
          write(o0 + j, it.P, racc[j], cacc[j], true);
        else
          write(o0 + j, it.Q, racc[j], racc[j], false);
      }
      if (!diag && m0 + j < kG) write(m0 + j, it.P, cacc[j], cacc[j], false);
    }
  }  // items
}

// out_o = (add ? add_o : 0) + alpha * sum of the item's partial slots
template <class T>
__global__ void __launch_bounds__(256) k_mv_reduce(int64_t n_out, const MvOut* __restrict__ outs,
                                                   const SubDev* __restrict__ subs, const T* __restrict__ partial,
                                                   T* __restrict__ out, const T* __restrict__ add_r, T alpha_r,
                                                   const T* __restrict__ add_c, T alpha_c, int nrhs,
                                                   const int* __restrict__ skip) {
  if (skip && *skip) return;
  if ((int64_t)blockIdx.x >= n_out) return;
  const MvOut w = outs[blockIdx.x];
  const SubDev q = subs[w.s];
  const bool crow = w.o >= q.kI + q.kG;
  const T* add = crow ? add_c : add_r;
  const T alpha = crow ? alpha_c : alpha_r;
  const int64_t base = (q.row_off + (int64_t)w.o * kNB) * nrhs;
  const int64_t stride = (int64_t)kNB * nrhs;
  // four consecutive elements per thread (a block holds 32 nrhs elements, a
  // multiple of 4, and every slot and output block starts on a multiple of 4)
  for (int e = 4 * threadIdx.x; e < kNB * nrhs; e += 4 * 256) {
    const T* pp = partial + (int64_t)w.slot0 * stride + e;
    T s[4] = {0, 0, 0, 0};
    // up to eight loads in flight before their adds (n is uniform: scalar
    // branches, no wasted loads); the sum keeps slot order
    for (int k = 0; k < w.nslot; k += 8) {
      const int n = min(8, w.nslot - k);
      T p[8][4];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (u < n) vload<T, 4>(pp + (int64_t)(k + u) * stride, p[u]);
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (u < n)
#pragma unroll
          for (int c = 0; c < 4; ++c) s[c] += p[u][c];
    }
    T v[4], a[4];
    if (add) vload<T, 4>(add + base + e, a);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      v[c] = alpha * s[c];
      if (add) v[c] += a[c];
    }
    vstore<T, 4>(out + base + e, v);
  }
}

// Nonzero count of every tile in [t0, t0 + n) (structural zeros of a
// nested-dissection-ordered factor and of its inverse are exact zeros).
template <class T>
__global__ void __launch_bounds__(256) k_tile_nnz(int64_t t0, int64_t n, const T* __restrict__ tiles,
                                                  int32_t* __restrict__ nnz, int32_t* __restrict__ qmask) {
  // one wave per tile: nonzeros of the tile (operand order), and per 16 x 16
  // quarter (bit 2 * row half + column half set when the quarter holds a
  // nonzero).  Lane l's 16-byte load k covers entries e = V (l + 64 k), whose
  // operand lane is l, so the quarter is 2 (e / 512) + l / 32: per-lane
  // counts and a shuffle sum per quarter, no atomics.
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= n) return;
  constexpr int V = 16 / sizeof(T);
  constexpr int L = kTile / (64 * V);  // loads per lane
  constexpr int P = 512 / (64 * V);    // loads per 512-entry half
  const int l = threadIdx.x & 63;
  typedef T vec_t __attribute__((ext_vector_type(V)));
  const vec_t* p = (const vec_t*)(tiles + (t0 + t) * kTile) + l;
  int a[2] = {0, 0};  // this lane's nonzeros in the row halves
#pragma unroll
  for (int k = 0; k < L; ++k) {
    const vec_t v = p[64 * k];
#pragma unroll
    for (int j = 0; j < V; ++j) a[k / P] += v[j] != (T)0;
  }
  // quarter 2 h + l / 32: sum over the lanes of each column half
  int c[4] = {l < 32 ? a[0] : 0, l < 32 ? 0 : a[0], l < 32 ? a[1] : 0, l < 32 ? 0 : a[1]};
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int q = 0; q < 4; ++q) c[q] += __shfl_xor(c[q], o);
  if (l == 0) {
    nnz[t] = c[0] + c[1] + c[2] + c[3];
    if (qmask) qmask[t] = (c[0] > 0) | (c[1] > 0) << 1 | (c[2] > 0) << 2 | (c[3] > 0) << 3;
  }
}

// Interface block of the local inverse K_rr^-1 = Linv_rr^T Linv_rr (the
// local inverses stored for the substitutions, Sec. III-C).  Linv_rr is lower
// triangular with Gamma ordered last in r, so the block is
// M = Linv_GG^T Linv_GG and the CG loop applies it in one symmetric product
// (k_symv).  One workgroup per tile (o, m), o >= m (interface tile indices):
//     M_om = sum_{k >= o} Linv_ko^T Linv_km,
// written in operand order to tile o(o+1)/2 + m of the subdomain's packed
// lower triangle (from tile m_off[s]).  Reads the row-major factor store.
template <class T>
__global__ void __launch_bounds__(256) k_schur_inv(int s0, const T* __restrict__ tiles,
                                                   const SubDev* __restrict__ subs,
                                                   const int64_t* __restrict__ m_off, T* __restrict__ msq,
                                                   const uint8_t* __restrict__ nzi) {
  const int sidx = s0 + blockIdx.y;
  const SubDev q = subs[sidx];
  const int p = blockIdx.x;  // p = o (o + 1) / 2 + m
  int o = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
  while ((o + 1) * (o + 2) / 2 <= p) ++o;
  while (o * (o + 1) / 2 > p) --o;
  const int m = p - o * (o + 1) / 2;
  if (o >= q.kG) return;
  __shared__ T A[kNB][kNB + 1];
  __shared__ T B[kNB][kNB + 1];
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, mb = w >> 1, nb = w & 1;
  typename Mfma<T>::acc_t acc = {0, 0, 0, 0};
  extern __shared__ uint16_t list[];
  __shared__ int wcnt[4];
  const int nn = chain_list(
      o, q.kG,
      [&](int k) { return nzi[tile_index(q, q.kI + k, q.kI + o)] && nzi[tile_index(q, q.kI + k, q.kI + m)]; },
      list, wcnt);
  chain_mma<T, true, false>(
      list, nn,
      [&](int k, const T*& ap, const T*& bp) {
        ap = tiles + tile_index(q, q.kI + k, q.kI + o) * kTile;  // Linv_ko (staged transposed)
        bp = tiles + tile_index(q, q.kI + k, q.kI + m) * kTile;  // Linv_km
      },
      A, B, acc);
  T* d = msq + (m_off[sidx] + (int64_t)o * (o + 1) / 2 + m) * kTile;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = mb * 16 + Mfma<T>::row(l, v), c = nb * 16 + (l & 15);
    d[swz<T>(r, c)] = acc[v];
  }
}

// Reorder every tile of a store from row-major into operand order, and
// write the operand-order transposed copy into tT.
template <class T>
__global__ void __launch_bounds__(256) k_pack_tiles(int64_t ntiles, T* __restrict__ tN, T* __restrict__ tT) {
  const int64_t t = blockIdx.x;
  if (t >= ntiles) return;
  __shared__ T a[kNB][kNB + 1];
  T* p = tN + t * kTile;
  for (int e = threadIdx.x; e < kTile; e += 256) a[e / kNB][e % kNB] = p[e];
  __syncthreads();
  T* q = tT + t * kTile;
  for (int e = threadIdx.x; e < kTile; e += 256) {
    const int r = e / kNB, c = e % kNB;
    p[swz<T>(r, c)] = a[r][c];
    q[swz<T>(r, c)] = a[c][r];
  }
}

// --------------------------------------------------------------------------
// Maps between the global unknown space, the multipliers and local blocks.
// --------------------------------------------------------------------------
// Local block rows <- owner split of a global FP64 vector [nint][nrhs]
// (src[row] = unknown id if this subdomain owns it, else -1).
template <class T>
__global__ void k_split(int64_t rows, const int32_t* __restrict__ src, const double* __restrict__ b,
                        T* __restrict__ w, int nrhs,
                        const int* __restrict__ skip) {
  if (skip && *skip) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * nrhs) return;
  int64_t row = i / nrhs;
  int r = (int)(i % nrhs);
  int32_t d = src[row];
  w[i] = d >= 0 ? (T)b[(int64_t)d * nrhs + r] : (T)0;
}

// v[row] = sign(row) * p[lam(row)] on listed rows (interface rows of every
// subdomain, padding rows included with lam = -1 -> 0): B_s^T p.
// With add: v[row] = add[row] - sign(row) * p[lam(row)] (the interface load
// left after the multipliers, y_G - B_s^T lambda).
template <class T>
__global__ void k_lambda_gather(int64_t n, const int64_t* __restrict__ rows, const int32_t* __restrict__ lam,
                                const double* __restrict__ p, T* __restrict__ v, int nrhs,
                                const int* __restrict__ skip, const T* __restrict__ add) {
  if (skip && *skip) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  int64_t k = i / nrhs;
  int r = (int)(i % nrhs);
  int32_t l = lam[k];
  double x = 0.0;
  if (l >= 0) x = (double)(l & 1 ? -1 : 1) * p[(int64_t)(l >> 1) * nrhs + r];
  const int64_t o = rows[k] * nrhs + r;
  v[o] = add ? (T)(add[o] - (T)x) : (T)x;
}

// F p = sum_s B_s u_s: each multiplier pulls its two copies (+lo, -hi).
template <class T>
__global__ void k_lambda_scatter(int64_t nlam, const int64_t* __restrict__ row0, const int64_t* __restrict__ row1,
                                 const T* __restrict__ u, double* __restrict__ out, int nrhs,
                                 const int* __restrict__ skip) {
  if (skip && *skip) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nlam * nrhs) return;
  int64_t l = i / nrhs;
  int r = (int)(i % nrhs);
  out[i] = (double)u[row0[l] * nrhs + r] - (double)u[row1[l] * nrhs + r];
}

// Coarse vector rows <- sum of the subdomain corner rows of each corner
// (fixed order) [+ add]; padding rows of the coarse block get 0.
template <class T>
__global__ void k_coarse_gather(int64_t ncrows, int64_t crow0, const int64_t* __restrict__ ptr,
                                const int64_t* __restrict__ rows, const T* __restrict__ x, T* __restrict__ y,
                                const T* __restrict__ add, int nrhs, const int* __restrict__ skip) {
  if (skip && *skip) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncrows * nrhs) return;
  int64_t c = i / nrhs;
  int r = (int)(i % nrhs);
  double s = 0.0;
  for (int64_t k = ptr[c]; k < ptr[c + 1]; ++k) s += (double)x[rows[k] * nrhs + r];
  int64_t o = (crow0 + c) * nrhs + r;
  if (add) s += (double)add[o];
  y[o] = (T)s;
}

// Subdomain corner rows <- scale * coarse solution (B_c z); crow = -1 -> 0.
template <class T>
__global__ void k_corner_scatter(int64_t n, const int64_t* __restrict__ rows, const int64_t* __restrict__ crow,
                                 const T* __restrict__ z, T* __restrict__ x, T scale, int nrhs,
                                 const int* __restrict__ skip) {
  if (skip && *skip) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  int64_t k = i / nrhs;
  int r = (int)(i % nrhs);
  int64_t c = crow[k];
  x[rows[k] * nrhs + r] = c >= 0 ? scale * z[c * nrhs + r] : (T)0;
}

// Vector forms of k_coarse_gather and k_corner_scatter: one thread per
// (row, group of V right-hand sides); the same sums in the same order.
template <class T, int V>
__global__ void k_coarse_gather_v(int64_t ncrows, int64_t crow0, const int64_t* __restrict__ ptr,
                                  const int64_t* __restrict__ rows, const T* __restrict__ x, T* __restrict__ y,
                                  const T* __restrict__ add, int nrhs, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int G = nrhs / V;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncrows * G) return;
  const int64_t c = i / G;
  const int q = (int)(i - c * G);
  double s[V];
#pragma unroll
  for (int w = 0; w < V; ++w) s[w] = 0.0;
  for (int64_t k = ptr[c]; k < ptr[c + 1]; ++k) {
    T a[V];
    vload<T, V>(x + rows[k] * nrhs + q * V, a);
#pragma unroll
    for (int w = 0; w < V; ++w) s[w] += (double)a[w];
  }
  const int64_t o = (crow0 + c) * nrhs + q * V;
  T out[V];
  if (add) {
    T a[V];
    vload<T, V>(add + o, a);
#pragma unroll
    for (int w = 0; w < V; ++w) s[w] += (double)a[w];
  }
#pragma unroll
  for (int w = 0; w < V; ++w) out[w] = (T)s[w];
  vstore<T, V>(y + o, out);
}

template <class T, int V>
__global__ void k_corner_scatter_v(int64_t n, const int64_t* __restrict__ rows, const int64_t* __restrict__ crow,
                                   const T* __restrict__ z, T* __restrict__ x, T scale, int nrhs,
                                   const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int G = nrhs / V;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * G) return;
  const int64_t k = i / G;
  const int q = (int)(i - k * G);
  const int64_t c = crow[k];
  T a[V];
  if (c >= 0) {
    vload<T, V>(z + c * nrhs + q * V, a);
#pragma unroll
    for (int w = 0; w < V; ++w) a[w] = scale * a[w];
  } else {
#pragma unroll
    for (int w = 0; w < V; ++w) a[w] = (T)0;
  }
  vstore<T, V>(x + rows[k] * nrhs + q * V, a);
}

// Vector forms of k_split, k_lambda_gather and k_collect: one thread per
// (row, group of V right-hand sides).
template <class T, int V>
__global__ void k_split_v(int64_t rows, const int32_t* __restrict__ src, const double* __restrict__ b,
                          T* __restrict__ w, int nrhs, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int G = nrhs / V;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * G) return;
  const int64_t row = i / G;
  const int q = (int)(i - row * G);
  const int32_t d = src[row];
  double x[V];
  T y[V];
  if (d >= 0) {
    vload<double, V>(b + (int64_t)d * nrhs + q * V, x);
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) x[v] = 0.0;
  }
#pragma unroll
  for (int v = 0; v < V; ++v) y[v] = (T)x[v];
  vstore<T, V>(w + row * nrhs + q * V, y);
}

template <class T, int V>
__global__ void k_lambda_gather_v(int64_t n, const int64_t* __restrict__ rows, const int32_t* __restrict__ lam,
                                  const double* __restrict__ p, T* __restrict__ v, int nrhs,
                                  const int* __restrict__ skip, const T* __restrict__ add) {
  if (skip && *skip) return;
  const int G = nrhs / V;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * G) return;
  const int64_t k = i / G;
  const int q = (int)(i - k * G);
  const int32_t l = lam[k];
  double x[V];
  T y[V];
  if (l >= 0) {
    vload<double, V>(p + (int64_t)(l >> 1) * nrhs + q * V, x);
  } else {
#pragma unroll
    for (int u = 0; u < V; ++u) x[u] = 0.0;
  }
  const double sg = l >= 0 && (l & 1) ? -1.0 : 1.0;
  const int64_t o = rows[k] * nrhs + q * V;
#pragma unroll
  for (int u = 0; u < V; ++u) y[u] = (T)(sg * x[u]);
  if (add) {
    T a[V];
    vload<T, V>(add + o, a);
#pragma unroll
    for (int u = 0; u < V; ++u) y[u] = (T)(a[u] - y[u]);
  }
  vstore<T, V>(v + o, y);
}

template <class T, int V>
__global__ void k_collect_v(int64_t nint, const int64_t* __restrict__ dsrc, const T* __restrict__ x,
                            double* __restrict__ e, int nrhs, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int G = nrhs / V;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nint * G) return;
  const int64_t d = i / G;
  const int q = (int)(i - d * G);
  T y[V];
  double o[V];
  vload<T, V>(x + dsrc[d] * nrhs + q * V, y);
#pragma unroll
  for (int u = 0; u < V; ++u) o[u] = (double)y[u];
  vstore<double, V>(e + d * nrhs + q * V, o);
}

// Global FP64 result of unknown d = the owner's copy (dsrc[d] = row).
template <class T>
__global__ void k_collect(int64_t nint, const int64_t* __restrict__ dsrc, const T* __restrict__ x,
                          double* __restrict__ e, int nrhs, const int* __restrict__ skip) {
  if (skip && *skip) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nint * nrhs) return;
  int64_t d = i / nrhs;
  int r = (int)(i % nrhs);
  e[i] = (double)x[dsrc[d] * nrhs + r];
}

// --------------------------------------------------------------------------
// Layout changes between caller arrays [nrhs][n_edges] and unknown-major
// [nint][nrhs].
// --------------------------------------------------------------------------
// Both are transposes through an LDS tile of 64 rows x nrhs, so global reads
// and writes are coalesced on both sides.
__global__ void __launch_bounds__(256) k_edges_to_int(int64_t nint, const int32_t* __restrict__ interior,
                                                      const double* __restrict__ src, int64_t ne,
                                                      double* __restrict__ dst, int nrhs, double scale) {
  __shared__ double tile[64][kMaxRhs + 1];
  const int64_t d0 = (int64_t)blockIdx.x * 64;
  const int tid = threadIdx.x;
  // all of a thread's loads (up to 64 kMaxRhs / 256) in flight before the
  // LDS stores
  constexpr int K = 64 * kMaxRhs / 256;
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = tid + 256 * k;
    const int r = e / 64, dl = e % 64;
    const int64_t d = d0 + dl;
    v[k] = e < 64 * nrhs && d < nint ? scale * src[(int64_t)r * ne + interior[d]] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int e = tid + 256 * k;
    if (e < 64 * nrhs) tile[e % 64][e / 64] = v[k];
  }
  __syncthreads();
  if (nrhs % 2 == 0) {
    // pairs of right-hand sides in 16-byte stores
    for (int e = tid; e < 32 * nrhs; e += 256) {
      const int dl = 2 * e / nrhs, r = 2 * e % nrhs;
      const int64_t d = d0 + dl;
      if (d < nint) *reinterpret_cast<double2*>(dst + d * nrhs + r) = make_double2(tile[dl][r], tile[dl][r + 1]);
    }
  } else {
    for (int e = tid; e < 64 * nrhs; e += 256) {
      const int dl = e / nrhs, r = e % nrhs;
      const int64_t d = d0 + dl;
      if (d < nint) dst[d * nrhs + r] = tile[dl][r];
    }
  }
}

__global__ void __launch_bounds__(256) k_int_to_edges(int64_t ne, const int32_t* __restrict__ dof,
                                                      const double* __restrict__ src, double* __restrict__ dst,
                                                      int nrhs, int accumulate, double scale) {
  __shared__ double tile[64][kMaxRhs + 1];
  const int64_t e0 = (int64_t)blockIdx.x * 64;
  const int tid = threadIdx.x;
  if (nrhs % 2 == 0) {
    // pairs of right-hand sides in 16-byte loads
    for (int k = tid; k < 32 * nrhs; k += 256) {
      const int el = 2 * k / nrhs, r = 2 * k % nrhs;
      const int64_t e = e0 + el;
      if (e < ne) {
        const int32_t d = dof[e];
        double2 x = make_double2(0.0, 0.0);
        if (d >= 0) x = *reinterpret_cast<const double2*>(src + (int64_t)d * nrhs + r);
        tile[el][r] = d >= 0 ? scale * x.x : 0.0;
        tile[el][r + 1] = d >= 0 ? scale * x.y : 0.0;
      }
    }
  } else {
    for (int k = tid; k < 64 * nrhs; k += 256) {
      const int el = k / nrhs, r = k % nrhs;
      const int64_t e = e0 + el;
      if (e < ne) {
        const int32_t d = dof[e];
        tile[el][r] = d >= 0 ? scale * src[(int64_t)d * nrhs + r] : 0.0;
      }
    }
  }
  __syncthreads();
  for (int k = tid; k < 64 * nrhs; k += 256) {
    const int r = k / 64, el = k % 64;
    const int64_t e = e0 + el;
    if (e >= ne) continue;
    const int64_t i = (int64_t)r * ne + e;
    if (accumulate) {
      if (dof[e] >= 0) dst[i] += tile[el][r];
    } else {
      dst[i] = tile[el][r];
    }
  }
}

// --------------------------------------------------------------------------
// K4: Newmark right-hand side and residuals with the global CSR of (T, S);
// ca = beta dt^2 (A = T + ca S), cb = (2 beta - 1) dt^2 (B1 = 2T + cb S).
//   mode 0: y = B1 x1 - A x2 - dt (j1 - j2)       (Newmark right-hand side)
//   mode 1: y = z - A x1, and y2 = T x1 if y2 != 0 (refinement residual;
//           T x1 feeds the Gauss-law check of the final iterate)
//   mode 2: y = B1 x1, y2 = A x1                  (adjoint application)
//   mode 3: y = T x1,  y2 = S x1                  (Gauss law, energy)
// One thread per (row, rhs); vectors [nint][nrhs].  Used for up to 4 RHS;
// k_csr_coop below computes the same for 5..32.
// --------------------------------------------------------------------------
// Rows are handed to XCDs in contiguous ranges (workgroup b runs on XCD
// b % 8): the column gathers of neighbouring rows then hit the same L2.
// The grid is a multiple of 8 workgroups.
__device__ __forceinline__ int64_t xcd_contiguous_block() {
  const int64_t per = gridDim.x / 8;
  return (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

__global__ void __launch_bounds__(256) k_csr(int mode, int64_t nint, const int64_t* __restrict__ rp,
                                             const int32_t* __restrict__ ci, const double2* __restrict__ v,
                                             const double* __restrict__ x1, const double* __restrict__ x2,
                                             const double* __restrict__ j1, const double* __restrict__ j2,
                                             const double* __restrict__ z, double dt, double ca, double cb,
                                             double* __restrict__ y, double* __restrict__ y2, int nrhs,
                                             const int* __restrict__ skip, double* __restrict__ y3) {
  if (skip && *skip) return;
  const int64_t i = xcd_contiguous_block() * blockDim.x + threadIdx.x;
  if (i >= nint * nrhs) return;
  const int64_t row = i / nrhs;
  const int r = (int)(i % nrhs);
  double t1 = 0.0, s1 = 0.0, t2 = 0.0, s2 = 0.0;
  const int64_t k0 = rp[row], k1 = rp[row + 1];
  // nonzeros in batches of 4: all index and value loads of a batch are
  // issued before the gathers (memory-level parallelism; 8 measured slower,
  // its register use halves the occupancy); the products are summed in
  // ascending nonzero order
  constexpr int B = 4;
  for (int64_t kb = k0; kb < k1; kb += B) {
    int32_t c[B];
    double2 av[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const bool ok = kb + u < k1;
      const int64_t k = ok ? kb + u : k0;  // in-bounds (the row is not empty here)
      const int32_t cv = ci[k];
      const double2 vv = v[k];
      c[u] = ok ? cv : -1;
      av[u] = ok ? vv : make_double2(0.0, 0.0);
    }
    // unconditional gathers (padding entries read column 0, then zeroed):
    // a masked load would branch and wait for all loads in flight
    double a[B], b[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int64_t o = (int64_t)(c[u] >= 0 ? c[u] : 0) * nrhs + r;
      const double va = x1[o];
      a[u] = c[u] >= 0 ? va : 0.0;
      if (mode == 0) {
        const double vb = x2[o];
        b[u] = c[u] >= 0 ? vb : 0.0;
      } else {
        b[u] = 0.0;
      }
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      if (c[u] < 0) break;
      t1 += av[u].x * a[u];
      s1 += av[u].y * a[u];
      if (mode == 0) {
        t2 += av[u].x * b[u];
        s2 += av[u].y * b[u];
      }
    }
  }
  if (mode == 0) {
    y[i] = (2.0 * t1 + cb * s1) - (t2 + ca * s2) - dt * (j1[i] - j2[i]);
  } else if (mode == 1) {
    y[i] = z[i] - (t1 + ca * s1);
    if (y2) y2[i] = t1;
    if (y3) y3[i] = s1;
  } else if (mode == 2) {
    y[i] = 2.0 * t1 + cb * s1;
    y2[i] = t1 + ca * s1;
  } else {
    y[i] = t1;
    y2[i] = s1;
  }
}

// Cooperative form of k_csr for 5..32 right-hand sides: the G lanes of a row
// (G = 8, 16 or 32 >= nrhs; lanes past nrhs only help with the loads) first
// load a batch of NB of the row's index/value pairs in one round trip and
// stage them in LDS; every lane of the row then reads them back as
// broadcasts and issues all gathers of the batch together (in chunks of 4
// up to the wave's longest row).  Rows of the edge
// matrices of tetrahedral meshes hold up to about 20 nonzeros, one batch of
// NB = 20.
// Each row lies inside one wavefront, so only the wave synchronises on LDS;
// the trip count of the batch loop is the wave's maximum, so the wave stays
// converged.  The products are summed in ascending nonzero order, as in
// k_csr.  MODE is k_csr's mode, fixed at compile time so that no gather
// sits in a branch.
template <int G, int NB, int MODE>
__global__ void __launch_bounds__(256) k_csr_coop(int64_t nint, const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci, const double2* __restrict__ v,
                                                  const double* __restrict__ x1, const double* __restrict__ x2,
                                                  const double* __restrict__ j1, const double* __restrict__ j2,
                                                  const double* __restrict__ z, double dt, double ca, double cb,
                                                  double* __restrict__ y, double* __restrict__ y2, int nrhs,
                                                  const int* __restrict__ skip, double* __restrict__ y3) {
  static_assert(G == 8 || G == 16 || G == 32, "lanes per row");
  if (skip && *skip) return;
  static_assert(NB % 4 == 0, "index reads of four");
  constexpr int E = (NB + G - 1) / G;  // staged nonzeros per lane
  constexpr int ROWS = 256 / G;         // rows per workgroup
  __shared__ int4 s_c[ROWS * NB / 4];
  __shared__ double2 s_v[ROWS * NB];
  const int64_t blk = xcd_contiguous_block();
  if (blk * (256 / G) >= nint) return;  // whole workgroup past the last row
  const int64_t i = blk * 256 + threadIdx.x;
  const int lr = (int)(i % G);
  const int64_t row_raw = i / G;
  const bool live = row_raw < nint && lr < nrhs;
  const int64_t row = row_raw < nint ? row_raw : nint - 1;
  const int rr = lr < nrhs ? lr : nrhs - 1;  // column of the gathers
  const int gb = ((int)threadIdx.x / G) * NB;  // this row's LDS slots
  int32_t* sc = reinterpret_cast<int32_t*>(s_c);
  const int64_t k0 = rp[row], k1 = rp[row + 1];
  int nbat = (int)((k1 - k0 + NB - 1) / NB);
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) nbat = max(nbat, __shfl_xor(nbat, off));
  double t1 = 0.0, s1 = 0.0, t2 = 0.0, s2 = 0.0;
  for (int bi = 0; bi < nbat; ++bi) {
    const int64_t kb = k0 + (int64_t)bi * NB;
    // nonzeros of this batch in the wave's longest row (uniform): chunks of
    // gathers past it are skipped
    int wcnt = (int)(k1 - kb < NB ? (k1 - kb > 0 ? k1 - kb : 0) : NB);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) wcnt = max(wcnt, __shfl_xor(wcnt, off));
    wcnt = __builtin_amdgcn_readfirstlane(wcnt);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int slot = e * G + lr;
      const int64_t k = kb + slot;
      const int64_t kc = k < k1 ? k : (k1 > k0 ? k0 : 0);  // in bounds (nnz > 0)
      const int32_t cv = ci[kc];
      const double2 vv = v[kc];
      // padding: the row's first column with a zero value (adds an exact
      // zero for finite x, and reads nothing outside the row's own columns)
      if (slot < NB) {
        sc[gb + slot] = cv;
        s_v[gb + slot] = k < k1 ? vv : make_double2(0.0, 0.0);
      }
    }
    wave_lds_sync();
    // gathers in chunks of 4 up to the wave's longest row, plain loads (no
    // select to wait on; each chunk reads its 4 columns from LDS just
    // before); all chunks go out before the first product waits.  MODE 0
    // gathers its second vector in a second round.
    auto gather = [&](const double* __restrict__ xv, double (&a)[NB]) {
#pragma unroll
      for (int u = 0; u < NB; ++u) a[u] = 0.0;
#pragma unroll
      for (int q = 0; q < NB / 4; ++q) {
        if (wcnt > 4 * q) {
          const int4 c4 = s_c[gb / 4 + q];
          a[4 * q] = xv[(int64_t)c4.x * nrhs + rr];
          a[4 * q + 1] = xv[(int64_t)c4.y * nrhs + rr];
          a[4 * q + 2] = xv[(int64_t)c4.z * nrhs + rr];
          a[4 * q + 3] = xv[(int64_t)c4.w * nrhs + rr];
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    };
    double a[NB];
    gather(x1, a);
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      const double2 vv = s_v[gb + u];
      t1 += vv.x * a[u];
      s1 += vv.y * a[u];
    }
    if constexpr (MODE == 0) {
      // a compiler-only fence that the first round's products feed: the
      // second round's loads stay after them (register pressure)
      __asm__ volatile("" : "+v"(t1), "+v"(s1)::"memory");
      gather(x2, a);
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const double2 vv = s_v[gb + u];
        t2 += vv.x * a[u];
        s2 += vv.y * a[u];
      }
    }
    wave_lds_sync();  // the next batch overwrites this row's slots
  }
  if (!live) return;
  const int64_t o = row * nrhs + lr;
  if constexpr (MODE == 0) {
    y[o] = (2.0 * t1 + cb * s1) - (t2 + ca * s2) - dt * (j1[o] - j2[o]);
  } else if constexpr (MODE == 1) {
    y[o] = z[o] - (t1 + ca * s1);
    if (y2) y2[o] = t1;
    if (y3) y3[o] = s1;
  } else if constexpr (MODE == 2) {
    y[o] = 2.0 * t1 + cb * s1;
    y2[o] = t1 + ca * s1;
  } else {
    y[o] = t1;
    y2[o] = s1;
  }
}

// Vector form of k_csr_coop: G lanes of a row with V right-hand sides each
// (nrhs = G V; G a power of two, so a row never straddles a wave).  A row's
// nonzeros are staged in LDS in batches of NB (the G lanes load NB / G each)
// and read back as broadcasts; each gather moves the V right-hand sides of
// one column (8V contiguous bytes), in chunks of 4 up to the wave's longest
// row.  Every right-hand side sums its products in ascending nonzero order,
// as in k_csr.  Modes as in k_csr.
template <int G, int V, int NB, int MODE>
__global__ void __launch_bounds__(256) k_csr_vec(int64_t nint, const int64_t* __restrict__ rp,
                                                 const int32_t* __restrict__ ci, const double2* __restrict__ v,
                                                 const double* __restrict__ x1, const double* __restrict__ x2,
                                                 const double* __restrict__ j1, const double* __restrict__ j2,
                                                 const double* __restrict__ z, double dt, double ca, double cb,
                                                 double* __restrict__ y, double* __restrict__ y2, int nrhs,
                                                 const int* __restrict__ skip, double* __restrict__ y3) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "lanes per row");
  static_assert(NB % G == 0 && NB % 4 == 0, "batch shape");
  if (skip && *skip) return;
  constexpr int ROWS = 256 / G;  // rows per workgroup
  constexpr int E = NB / G;      // staged nonzeros per lane
  __shared__ int32_t s_c[ROWS * NB];
  __shared__ double2 s_v[ROWS * NB];
  const int64_t blk = xcd_contiguous_block();
  if (blk * ROWS >= nint) return;  // whole workgroup past the last row
  const int lr = (int)threadIdx.x % G;
  const int64_t row_raw = blk * ROWS + (int)threadIdx.x / G;
  const bool live = row_raw < nint;
  const int64_t row = live ? row_raw : nint - 1;
  const int gb = ((int)threadIdx.x / G) * NB;  // this row's LDS slots
  const int64_t xo = (int64_t)lr * V;            // this lane's right-hand sides
  const int64_t k0 = rp[row], k1 = rp[row + 1];
  int nbat = (int)((k1 - k0 + NB - 1) / NB);
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) nbat = max(nbat, __shfl_xor(nbat, off));
  double t1[V], s1[V], t2[V], s2[V];
#pragma unroll
  for (int w = 0; w < V; ++w) t1[w] = s1[w] = t2[w] = s2[w] = 0.0;
  for (int bi = 0; bi < nbat; ++bi) {
    const int64_t kb = k0 + (int64_t)bi * NB;
    int wcnt = (int)(k1 - kb < NB ? (k1 - kb > 0 ? k1 - kb : 0) : NB);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) wcnt = max(wcnt, __shfl_xor(wcnt, off));
    wcnt = __builtin_amdgcn_readfirstlane(wcnt);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int slot = e * G + lr;
      const int64_t k = kb + slot;
      const int64_t kc = k < k1 ? k : (k1 > k0 ? k0 : 0);  // in bounds (nnz > 0)
      const int32_t cv = ci[kc];
      const double2 vv = v[kc];
      // padding: the row's first column with a zero value
      s_c[gb + slot] = cv;
      s_v[gb + slot] = k < k1 ? vv : make_double2(0.0, 0.0);
    }
    wave_lds_sync();
    auto run = [&](const double* __restrict__ xv, double (&tt)[V], double (&ss)[V]) {
      double a[NB][V];
#pragma unroll
      for (int q = 0; q < NB / 4; ++q) {
        if (wcnt > 4 * q) {
#pragma unroll
          for (int u = 4 * q; u < 4 * q + 4; ++u) vload<double, V>(xv + (int64_t)s_c[gb + u] * nrhs + xo, a[u]);
        } else {
#pragma unroll
          for (int u = 4 * q; u < 4 * q + 4; ++u)
#pragma unroll
            for (int w = 0; w < V; ++w) a[u][w] = 0.0;
        }
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < NB; ++u) {
        const double2 vv = s_v[gb + u];
#pragma unroll
        for (int w = 0; w < V; ++w) {
          tt[w] += vv.x * a[u][w];
          ss[w] += vv.y * a[u][w];
        }
      }
    };
    run(x1, t1, s1);
    if constexpr (MODE == 0) {
      __asm__ volatile("" ::: "memory");
      run(x2, t2, s2);
    }
    wave_lds_sync();  // the next batch overwrites this row's slots
  }
  if (!live) return;
  const int64_t o = row * nrhs + xo;
  double r0[V], r1[V], r2[V];
  if constexpr (MODE == 0) {
    double a1[V], a2[V];
    vload<double, V>(j1 + o, a1);
    vload<double, V>(j2 + o, a2);
#pragma unroll
    for (int w = 0; w < V; ++w) r0[w] = (2.0 * t1[w] + cb * s1[w]) - (t2[w] + ca * s2[w]) - dt * (a1[w] - a2[w]);
    vstore<double, V>(y + o, r0);
  } else if constexpr (MODE == 1) {
    double zz[V];
    vload<double, V>(z + o, zz);
#pragma unroll
    for (int w = 0; w < V; ++w) r0[w] = zz[w] - (t1[w] + ca * s1[w]);
    vstore<double, V>(y + o, r0);
    if (y2) vstore<double, V>(y2 + o, t1);
    if (y3) vstore<double, V>(y3 + o, s1);
  } else if constexpr (MODE == 2) {
#pragma unroll
    for (int w = 0; w < V; ++w) {
      r1[w] = 2.0 * t1[w] + cb * s1[w];
      r2[w] = t1[w] + ca * s1[w];
    }
    vstore<double, V>(y + o, r1);
    vstore<double, V>(y2 + o, r2);
  } else {
    vstore<double, V>(y + o, t1);
    vstore<double, V>(y2 + o, s1);
  }
}

// Newmark load from stored products (the resident step): with te = T e,
// se = S e of e^n (0) and e^{n-1} (1),
//   y = (2 T e^n + cb S e^n) - (T e^{n-1} + ca S e^{n-1}) - dt (J^{n+1/2} - J^{n-1/2}),
// the same expression, in the same order, as mode 0 of k_csr / k_csr_coop.
__global__ void __launch_bounds__(256) k_newmark_load(int64_t n, const double* __restrict__ te0,
                                                      const double* __restrict__ se0, const double* __restrict__ te1,
                                                      const double* __restrict__ se1, const double* __restrict__ j1,
                                                      const double* __restrict__ j0, double dt, double ca, double cb,
                                                      double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  y[i] = (2.0 * te0[i] + cb * se0[i]) - (te1[i] + ca * se1[i]) - dt * (j1[i] - j0[i]);
}

// --------------------------------------------------------------------------
// K8: conjugate gradients on the interface system, per right-hand side.
// Dot products: fixed-order two-stage reductions (deterministic).
// --------------------------------------------------------------------------
constexpr int kDotBlocks = 1024;

__global__ void __launch_bounds__(256) k_dot_partial(int64_t n, const double* __restrict__ x,
                                                     const double* __restrict__ y, int nrhs,
                                                     double* __restrict__ partial, const int* __restrict__ skip) {
  if (skip && *skip) return;
  // block b sums rows b, b + B, ... for every rhs; layout [n][nrhs]
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int lanes_per_rhs = 256 / nrhs;  // nrhs divides 256 (powers of two) or nrhs <= 256
  const int r = tid % nrhs;
  const int lane = tid / nrhs;
  double s = 0.0;
  if (lane < lanes_per_rhs) {
    for (int64_t row = (int64_t)blockIdx.x * lanes_per_rhs + lane; row < n;
         row += (int64_t)gridDim.x * lanes_per_rhs)
      s += x[row * nrhs + r] * y[row * nrhs + r];
  }
  red[tid] = s;
  __syncthreads();
  if (tid < nrhs) {
    double t = 0.0;
    for (int l = 0; l < lanes_per_rhs; ++l) t += red[l * nrhs + tid];
    partial[blockIdx.x * kMaxRhs + tid] = t;
  }
}

// Vector form of k_dot_partial: V right-hand sides per lane (nrhs a
// multiple of V), one 8V-byte load of each vector per row.
template <int V>
__global__ void __launch_bounds__(256) k_dot_partial_v(int64_t n, const double* __restrict__ x,
                                                       const double* __restrict__ y, int nrhs,
                                                       double* __restrict__ partial, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int G = nrhs / V, lpr = 256 / G;
  const int tid = threadIdx.x, q = tid % G, lane = tid / G;
  double s[V];
#pragma unroll
  for (int w = 0; w < V; ++w) s[w] = 0.0;
  if (lane < lpr) {
    for (int64_t row = (int64_t)blockIdx.x * lpr + lane; row < n; row += (int64_t)gridDim.x * lpr) {
      double a[V], b[V];
      vload<double, V>(x + row * nrhs + q * V, a);
      vload<double, V>(y + row * nrhs + q * V, b);
#pragma unroll
      for (int w = 0; w < V; ++w) s[w] += a[w] * b[w];
    }
  }
  block_rhs_sum_v<V>(s, nrhs, lpr, partial);
}

// Block-level sum of per-thread values s (thread layout tid = lane*nrhs + r)
// into partial[blockIdx.x][r].
__device__ __forceinline__ void block_rhs_sum(double s, int nrhs, int lanes_per_rhs, double* __restrict__ partial) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  red[tid] = s;
  __syncthreads();
  if (tid < nrhs) {
    double t = 0.0;
    for (int l = 0; l < lanes_per_rhs; ++l) t += red[l * nrhs + tid];
    partial[blockIdx.x * kMaxRhs + tid] = t;
  }
}

// F p = sum_s B_s u_s (each multiplier pulls its two copies, + lo, - hi),
// fused with the block partials of p . Fp.
// u2 (may be null) is added to u first, in T: the local response split
// over two buffers (the symmetric product and the corner coupling, written
// by different streams).
template <class T>
__global__ void __launch_bounds__(256) k_scatter_dot(int64_t nlam, const int64_t* __restrict__ row0,
                                                     const int64_t* __restrict__ row1, const T* __restrict__ u,
                                                     const T* __restrict__ u2, double* __restrict__ Fp,
                                                     const double* __restrict__ p, int nrhs,
                                                     double* __restrict__ partial, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int lpr = 256 / nrhs;
  const int tid = threadIdx.x, r = tid % nrhs, lane = tid / nrhs;
  // RU multipliers of the lane's grid-stride sequence in flight at once
  // (indices, then gathers; reads past the end are clamped and not used);
  // the dot is summed in the order of the plain loop
  constexpr int RU = 4;
  const int64_t stride = (int64_t)gridDim.x * lpr;
  double s = 0.0;
  if (lane < lpr) {
    for (int64_t l0 = (int64_t)blockIdx.x * lpr + lane; l0 < nlam; l0 += RU * stride) {
      int64_t a[RU], b[RU], lc[RU];
#pragma unroll
      for (int j = 0; j < RU; ++j) {
        const int64_t l = l0 + j * stride;
        lc[j] = l < nlam ? l : nlam - 1;
        a[j] = row0[lc[j]] * nrhs + r;
        b[j] = row1[lc[j]] * nrhs + r;
      }
      T ua[RU], ub[RU];
      double pv[RU];
#pragma unroll
      for (int j = 0; j < RU; ++j) {
        ua[j] = u2 ? (T)(u[a[j]] + u2[a[j]]) : u[a[j]];
        ub[j] = u2 ? (T)(u[b[j]] + u2[b[j]]) : u[b[j]];
        pv[j] = p ? p[lc[j] * nrhs + r] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < RU; ++j) {
        const int64_t l = l0 + j * stride;
        if (l < nlam) {
          const double f = (double)ua[j] - (double)ub[j];
          Fp[l * nrhs + r] = f;
          if (p) s += pv[j] * f;
        }
      }
    }
  }
  block_rhs_sum(s, nrhs, lpr, partial);
}

// Vector form of k_scatter_dot (V right-hand sides per lane).
template <class T, int V>
__global__ void __launch_bounds__(256) k_scatter_dot_v(int64_t nlam, const int64_t* __restrict__ row0,
                                                       const int64_t* __restrict__ row1, const T* __restrict__ u,
                                                       const T* __restrict__ u2, double* __restrict__ Fp,
                                                       const double* __restrict__ p, int nrhs,
                                                       double* __restrict__ partial, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int G = nrhs / V, lpr = 256 / G;
  const int tid = threadIdx.x, q = tid % G, lane = tid / G;
  constexpr int RU = 4;
  const int64_t stride = (int64_t)gridDim.x * lpr;
  double s[V];
#pragma unroll
  for (int v = 0; v < V; ++v) s[v] = 0.0;
  if (lane < lpr) {
    for (int64_t l0 = (int64_t)blockIdx.x * lpr + lane; l0 < nlam; l0 += RU * stride) {
      int64_t a[RU], b[RU], lc[RU];
#pragma unroll
      for (int j = 0; j < RU; ++j) {
        const int64_t l = l0 + j * stride;
        lc[j] = l < nlam ? l : nlam - 1;
        a[j] = row0[lc[j]] * nrhs + q * V;
        b[j] = row1[lc[j]] * nrhs + q * V;
      }
      T ua[RU][V], ub[RU][V], ta[RU][V], tb[RU][V];
      double pv[RU][V];
#pragma unroll
      for (int j = 0; j < RU; ++j) {
        vload<T, V>(u + a[j], ua[j]);
        vload<T, V>(u + b[j], ub[j]);
        if (u2) {
          vload<T, V>(u2 + a[j], ta[j]);
          vload<T, V>(u2 + b[j], tb[j]);
        }
        if (p) {
          vload<double, V>(p + lc[j] * nrhs + q * V, pv[j]);
        } else {
#pragma unroll
          for (int v = 0; v < V; ++v) pv[j][v] = 0.0;
        }
      }
#pragma unroll
      for (int j = 0; j < RU; ++j) {
        const int64_t l = l0 + j * stride;
        if (l < nlam) {
          double f[V];
#pragma unroll
          for (int v = 0; v < V; ++v) {
            const T x0 = u2 ? (T)(ua[j][v] + ta[j][v]) : ua[j][v];
            const T x1 = u2 ? (T)(ub[j][v] + tb[j][v]) : ub[j][v];
            f[v] = (double)x0 - (double)x1;
            if (p) s[v] += pv[j][v] * f[v];
          }
          vstore<double, V>(Fp + l * nrhs + q * V, f);
        }
      }
    }
  }
  block_rhs_sum_v<V>(s, nrhs, lpr, partial);
}

struct CgState {
  double rr[kMaxRhs];      // current r.r
  double rz[kMaxRhs];      // current r.z (z = preconditioned r; r.r without a preconditioner)
  double rr0[kMaxRhs];     // d.d (relative tolerance reference)
  double alpha[kMaxRhs];
  double beta[kMaxRhs];
  int active[kMaxRhs];
  int iters[kMaxRhs];
  int done;                // all right-hand sides converged (or broke down)
  int breakdown;
};

// stage: 0 = init (rr = rr0 = rz = sum A), 1 = alpha = rz / (sum A = p.Fp),
//        2 = beta (sum A = new r.z, sum B = new r.r), 3 = warm start (rr = rz =
//        sum A, convergence flags only), 4 = preconditioned start (rz = sum A)
// One workgroup of kScalarThreads threads (the first level of the sum is
// kDotBlocks / lanes deep; with 1024 threads a short chain of L2 loads).
constexpr int kScalarThreads = 1024;
__global__ void __launch_bounds__(kScalarThreads) k_cg_scalar(int stage, int nrhs, const double* __restrict__ partial,
                                                              const double* __restrict__ partial_b,
                                                              CgState* __restrict__ st, double tol,
                                                              const int* __restrict__ gate) {
  if (gate && *gate) return;
  if (stage != 0 && st->done) return;
  const int r = threadIdx.x;
  __shared__ int any_active;
  if (r == 0) any_active = 0;
  __syncthreads();
  // fixed-order two-level sum of the block partials: thread t sums blocks
  // t/nrhs, t/nrhs + L, ... of rhs t%nrhs, then lanes are added in order
  __shared__ double part[kScalarThreads];
  auto total = [&](const double* pa) -> double {
    const int t = threadIdx.x, lpr = blockDim.x / nrhs, rr = t % nrhs, ln = t / nrhs;
    double a = 0.0;
    if (ln < lpr) {
#pragma unroll 4
      for (int b = ln; b < kDotBlocks; b += lpr) a += pa[b * kMaxRhs + rr];
    }
    part[t] = a;
    __syncthreads();
    double v = 0.0;
    if (t < nrhs)
      for (int l = 0; l < lpr; ++l) v += part[l * nrhs + t];
    __syncthreads();
    return v;
  };
  const double s = total(partial);
  const double sb = stage == 2 ? total(partial_b) : 0.0;
  if (stage == 0 && r == 0) st->breakdown = 0;  // stage 0 resets the whole state
  if (r < nrhs) {
    if (stage == 0) {
      st->rr[r] = s;
      st->rr0[r] = s;
      st->rz[r] = s;
      st->iters[r] = 0;
      st->active[r] = s > 0.0 ? 1 : 0;
      st->alpha[r] = 0.0;
      st->beta[r] = 0.0;
    } else if (stage == 3) {
      st->rr[r] = s;
      st->rz[r] = s;
      st->beta[r] = 0.0;
      if (st->active[r] && s <= tol * tol * st->rr0[r]) st->active[r] = 0;
    } else if (stage == 4) {
      st->rz[r] = s;
    } else if (stage == 1) {
      if (st->active[r]) {
        if (!(s > 0.0) || !isfinite(s)) {
          st->active[r] = 0;
          st->alpha[r] = 0.0;
          atomicOr(&st->breakdown, 1);
        } else {
          st->alpha[r] = st->rz[r] / s;
        }
      } else {
        st->alpha[r] = 0.0;
      }
    } else {
      if (st->active[r]) {
        st->iters[r] += 1;
        st->beta[r] = s / st->rz[r];
        st->rz[r] = s;
        st->rr[r] = sb;
        if (!(sb <= tol * tol * st->rr0[r])) {
          // keep iterating (also on NaN: caught by the caller's cap)
        } else {
          st->active[r] = 0;
        }
      } else {
        st->beta[r] = 0.0;
      }
    }
    if (st->active[r]) atomicOr(&any_active, 1);
  }
  __syncthreads();
  if (r == 0) st->done = any_active ? 0 : 1;
}

// lambda += alpha p ; r -= alpha Fp, fused with the block partials of r . r
__global__ void __launch_bounds__(256) k_cg_xr_dot(int64_t n, int nrhs, const CgState* __restrict__ st,
                                                   const double* __restrict__ p, const double* __restrict__ Fp,
                                                   double* __restrict__ lam, double* __restrict__ res,
                                                   double* __restrict__ partial) {
  if (st->done) return;
  const int lpr = 256 / nrhs;
  const int tid = threadIdx.x, r = tid % nrhs, lane = tid / nrhs;
  double s = 0.0;
  if (lane < lpr) {
    const double a = st->alpha[r];
    for (int64_t l = (int64_t)blockIdx.x * lpr + lane; l < n; l += (int64_t)gridDim.x * lpr) {
      const int64_t i = l * nrhs + r;
      lam[i] += a * p[i];
      const double rv = res[i] - a * Fp[i];
      res[i] = rv;
      s += rv * rv;
    }
  }
  block_rhs_sum(s, nrhs, lpr, partial);
}

// lambda += alpha p ; r -= alpha Fp   (alpha = 0 for inactive rhs)
__global__ void k_cg_xr(int64_t n, int nrhs, const CgState* __restrict__ st, const double* __restrict__ p,
                        const double* __restrict__ Fp, double* __restrict__ lam, double* __restrict__ res) {
  if (st->done) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * nrhs) return;
  const double a = st->alpha[(int)(i % nrhs)];
  lam[i] += a * p[i];
  res[i] -= a * Fp[i];
}

// Vector form of k_cg_xr: V consecutive entries (of one multiplier row) per
// thread, nrhs a multiple of V.
template <int V>
__global__ void k_cg_xr_v(int64_t n, int nrhs, const CgState* __restrict__ st, const double* __restrict__ p,
                          const double* __restrict__ Fp, double* __restrict__ lam, double* __restrict__ res) {
  if (st->done) return;
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * V;
  if (i >= n * nrhs) return;
  const int r0 = (int)(i % nrhs);
  double pv[V], fv[V], lv[V], rv[V];
  vload<double, V>(p + i, pv);
  vload<double, V>(Fp + i, fv);
  vload<double, V>(lam + i, lv);
  vload<double, V>(res + i, rv);
#pragma unroll
  for (int w = 0; w < V; ++w) {
    const double a = st->alpha[r0 + w];
    lv[w] += a * pv[w];
    rv[w] -= a * fv[w];
  }
  vstore<double, V>(lam + i, lv);
  vstore<double, V>(res + i, rv);
}

// z = K_lam r (the lumped preconditioner, CSR in multiplier space), fused
// with the block partials of r.z (partial) and r.r (partial_b).
template <int RU, int KB>
__global__ void __launch_bounds__(256, 4) k_lam_precond(int64_t nlam, const int64_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, const double* __restrict__ val,
                                                     const double* __restrict__ res, double* __restrict__ z, int nrhs,
                                                     double* __restrict__ partial, double* __restrict__ partial_b,
                                                     const int* __restrict__ skip) {
  if (skip && *skip) return;
  // Each lane keeps RU rows of its grid-stride sequence in flight and loads
  // up to KB nonzeros of each before the gathers (unconditional loads from
  // clamped indices; padding entries are zeroed at the products), so a pass
  // costs three round trips for RU rows.  Rows, and the nonzeros in a row,
  // are summed in the order of the plain loop.
  const int lpr = 256 / nrhs;
  const int tid = threadIdx.x, r = tid % nrhs, lane = tid / nrhs;
  const int64_t stride = (int64_t)gridDim.x * lpr;
  double sz = 0.0, sr = 0.0;
  if (lane < lpr) {
    for (int64_t l0 = (int64_t)blockIdx.x * lpr + lane; l0 < nlam; l0 += RU * stride) {
      int64_t ka[RU], kz[RU];
      double rv[RU], acc[RU];
#pragma unroll
      for (int j = 0; j < RU; ++j) {
        const int64_t l = l0 + j * stride;
        const int64_t lc = l < nlam ? l : nlam - 1;
        const int64_t a0 = rp[lc], a1 = rp[lc + 1];
        const double x = res[lc * nrhs + r];
        ka[j] = a0;
        kz[j] = l < nlam ? a1 : a0;  // rows past the end are empty
        rv[j] = x;
        acc[j] = 0.0;
      }
      int nb = 0;
#pragma unroll
      for (int j = 0; j < RU; ++j) nb = max(nb, (int)((kz[j] - ka[j] + KB - 1) / KB));
      for (int bi = 0; bi < nb; ++bi) {
        int32_t c[RU][KB];
        double v[RU][KB], x[RU][KB];
#pragma unroll
        for (int j = 0; j < RU; ++j)
#pragma unroll
          for (int u = 0; u < KB; ++u) {
            const int64_t k = ka[j] + (int64_t)bi * KB + u;
            const int64_t kc = k < kz[j] ? k : 0;  // in bounds (the matrix is not empty here)
            c[j][u] = ci[kc];
            v[j][u] = val[kc];
          }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < RU; ++j)
#pragma unroll
          for (int u = 0; u < KB; ++u) x[j][u] = res[(int64_t)c[j][u] * nrhs + r];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < RU; ++j)
#pragma unroll
          for (int u = 0; u < KB; ++u) {
            const int64_t k = ka[j] + (int64_t)bi * KB + u;
            acc[j] += (k < kz[j] ? v[j][u] : 0.0) * x[j][u];
          }
      }
#pragma unroll
      for (int j = 0; j < RU; ++j) {
        const int64_t l = l0 + j * stride;
        if (l < nlam) {
          z[l * nrhs + r] = acc[j];
          sz += rv[j] * acc[j];
          sr += rv[j] * rv[j];
        }
      }
    }
  }
  block_rhs_sum(sz, nrhs, lpr, partial);
  __syncthreads();
  block_rhs_sum(sr, nrhs, lpr, partial_b);
}

// Vector form of k_lam_precond: V consecutive right-hand sides per lane
// (nrhs a multiple of V, G = nrhs / V lanes per row), so that the index and
// value loads of a nonzero are shared by G lanes instead of nrhs and each
// gather moves 8V contiguous bytes.  RU rows per lane in flight, their
// nonzeros in batches of KB, as in k_lam_precond; each right-hand side's
// rows and nonzeros are summed in the order of the plain loop, the block
// partials over lanes in lane order.
template <int RU, int KB, int V>
__global__ void __launch_bounds__(256, 4) k_lam_precond_v(int64_t nlam, const int64_t* __restrict__ rp,
                                                       const int32_t* __restrict__ ci, const double* __restrict__ val,
                                                       const double* __restrict__ res, double* __restrict__ z,
                                                       int nrhs, double* __restrict__ partial,
                                                       double* __restrict__ partial_b, const int* __restrict__ skip) {
  static_assert(V == 2 || V == 4, "right-hand sides per lane");
  if (skip && *skip) return;
  const int G = nrhs / V;
  const int lpr = 256 / G;
  const int tid = threadIdx.x, q = tid % G, lane = tid / G;
  const int64_t stride = (int64_t)gridDim.x * lpr;
  double sz[V], sr[V];
#pragma unroll
  for (int v = 0; v < V; ++v) sz[v] = sr[v] = 0.0;
  auto load = [&](const double* a, double (&o)[V]) { vload<double, V>(a, o); };
  if (lane < lpr) {
    for (int64_t l0 = (int64_t)blockIdx.x * lpr + lane; l0 < nlam; l0 += RU * stride) {
      int64_t ka[RU], kz[RU];
      double rv[RU][V], acc[RU][V];
#pragma unroll
      for (int j = 0; j < RU; ++j) {
        const int64_t l = l0 + j * stride;
        const int64_t lc = l < nlam ? l : nlam - 1;
        const int64_t a0 = rp[lc], a1 = rp[lc + 1];
        load(res + lc * nrhs + q * V, rv[j]);
        ka[j] = a0;
        kz[j] = l < nlam ? a1 : a0;  // rows past the end are empty
#pragma unroll
        for (int v = 0; v < V; ++v) acc[j][v] = 0.0;
      }
      int nb = 0;
#pragma unroll
      for (int j = 0; j < RU; ++j) nb = max(nb, (int)((kz[j] - ka[j] + KB - 1) / KB));
      for (int bi = 0; bi < nb; ++bi) {
        int32_t c[RU][KB];
        double w[RU][KB], x[RU][KB][V];
#pragma unroll
        for (int j = 0; j < RU; ++j)
#pragma unroll
          for (int u = 0; u < KB; ++u) {
            const int64_t k = ka[j] + (int64_t)bi * KB + u;
            const int64_t kc = k < kz[j] ? k : 0;  // in bounds (the matrix is not empty here)
            c[j][u] = ci[kc];
            w[j][u] = val[kc];
          }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < RU; ++j)
#pragma unroll
          for (int u = 0; u < KB; ++u) load(res + (int64_t)c[j][u] * nrhs + q * V, x[j][u]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int j = 0; j < RU; ++j)
#pragma unroll
          for (int u = 0; u < KB; ++u) {
            const int64_t k = ka[j] + (int64_t)bi * KB + u;
            const double wv = k < kz[j] ? w[j][u] : 0.0;
#pragma unroll
            for (int v = 0; v < V; ++v) acc[j][v] += wv * x[j][u][v];
          }
      }
#pragma unroll
      for (int j = 0; j < RU; ++j) {
        const int64_t l = l0 + j * stride;
        if (l < nlam) {
          vstore<double, V>(z + l * nrhs + q * V, acc[j]);
#pragma unroll
          for (int v = 0; v < V; ++v) {
            sz[v] += rv[j][v] * acc[j][v];
            sr[v] += rv[j][v] * rv[j][v];
          }
        }
      }
    }
  }
  block_rhs_sum_v<V>(sz, nrhs, lpr, partial);
  block_rhs_sum_v<V>(sr, nrhs, lpr, partial_b);
}

// p' = base + beta p for the RHS still active after the beta stage (p kept
// otherwise; base = z, or r without a preconditioner), once per multiplier
// (coalesced reads and writes of the multiplier vectors), then v = B_s^T p'
// scattered to its two interface rows, + in the lower subdomain (row0) and
// - in the higher (row1).  p alternates between two buffers.  Interface
// rows without a multiplier (padding) are not written: they keep the zeros
// of the solve's first gather (k_lambda_gather).
template <class T>
__global__ void k_cg_p_scatter(int64_t nlam, const int64_t* __restrict__ row0, const int64_t* __restrict__ row1,
                               int nrhs, const CgState* __restrict__ st, const double* __restrict__ base,
                               const double* __restrict__ pcur, double* __restrict__ pnext, T* __restrict__ v) {
  if (st->done) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nlam * nrhs) return;
  const int64_t l = i / nrhs;
  const int r = (int)(i - l * nrhs);
  const double pn = st->active[r] ? base[i] + st->beta[r] * pcur[i] : pcur[i];
  pnext[i] = pn;
  v[row0[l] * nrhs + r] = (T)pn;
  v[row1[l] * nrhs + r] = (T)(-pn);
}

// Vector form of k_cg_p_scatter: one thread per (multiplier, group of V
// right-hand sides).
template <class T, int V>
__global__ void k_cg_p_scatter_v(int64_t nlam, const int64_t* __restrict__ row0, const int64_t* __restrict__ row1,
                                 int nrhs, const CgState* __restrict__ st, const double* __restrict__ base,
                                 const double* __restrict__ pcur, double* __restrict__ pnext, T* __restrict__ v) {
  if (st->done) return;
  const int G = nrhs / V;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nlam * G) return;
  const int64_t l = i / G;
  const int q = (int)(i - l * G);
  const int64_t o = l * nrhs + q * V;
  double bv[V], pc[V], pn[V];
  vload<double, V>(base + o, bv);
  vload<double, V>(pcur + o, pc);
  T yp[V], ym[V];
#pragma unroll
  for (int u = 0; u < V; ++u) {
    const int r = q * V + u;
    pn[u] = st->active[r] ? bv[u] + st->beta[r] * pc[u] : pc[u];
    yp[u] = (T)pn[u];
    ym[u] = (T)(-pn[u]);
  }
  vstore<double, V>(pnext + o, pn);
  vstore<T, V>(v + row0[l] * nrhs + q * V, yp);
  vstore<T, V>(v + row1[l] * nrhs + q * V, ym);
}

__global__ void k_extrap(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                         double* __restrict__ y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = 2.0 * a[i] - b[i];
}

__global__ void k_axpy(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y,
                       const int* __restrict__ skip) {
  if (skip && *skip) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

// y = x, and a typed zero fill, both gated (used in place of memcpy /
// memset so that a captured step can skip them)
__global__ void k_copy(int64_t n, const double* __restrict__ x, double* __restrict__ y,
                       const int* __restrict__ skip) {
  if (skip && *skip) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}

template <class T>
__global__ void k_zero(int64_t n, T* __restrict__ y, const int* __restrict__ skip) {
  if (skip && *skip) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (T)0;
}

// y[0 .. n16) = 0 in 16-byte stores (grid-stride)
__global__ void k_clear16(int64_t n16, uint4* __restrict__ y) {
  const uint4 z = {0u, 0u, 0u, 0u};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = z;
}

__global__ void k_set_int(int* __restrict__ p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void k_fill(int64_t n, double v, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = v;
}

// dv = (a - b) * s, av = (a + b) / 2 (the energy's difference and average)
__global__ void k_diff_avg(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double s,
                           double* __restrict__ dv, double* __restrict__ av) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = a[i], y = b[i];
  dv[i] = (x - y) * s;
  av[i] = 0.5 * (x + y);
}

__global__ void k_sub(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a[i] - b[i];
}

// --------------------------------------------------------------------------
// Adjoint: eps_bar[k] -= sum_r g_r . T_k acc_r over the tet's interior
// edges (T_k = unit-eps element mass), acc = e^{n+1} - 2 e^n + e^{n-1}.
// --------------------------------------------------------------------------
__global__ void k_eps_bar(int64_t nt, const int32_t* __restrict__ tdof, const double* __restrict__ Te,
                          const double* __restrict__ g, const double* __restrict__ acc, int nrhs,
                          double* __restrict__ eps_bar) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nt) return;
  int32_t d[6];
  for (int a = 0; a < 6; ++a) d[a] = tdof[6 * t + a];
  double s = 0.0;
  for (int r = 0; r < nrhs; ++r)
    for (int a = 0; a < 6; ++a) {
      if (d[a] < 0) continue;
      double ga = g[(int64_t)d[a] * nrhs + r];
      double u = 0.0;
      for (int b = 0; b < 6; ++b)
        if (d[b] >= 0) u += Te[36 * t + 6 * a + b] * acc[(int64_t)d[b] * nrhs + r];
      s += ga * u;
    }
  eps_bar[t] -= s;
}

__global__ void k_second_diff(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                              const double* __restrict__ c, double* __restrict__ y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a[i] - 2.0 * b[i] + (c ? c[i] : 0.0);
}

// --------------------------------------------------------------------------
// K10: discrete Gauss law and energy.
// Node charge: q[r][v] += dt * sum_{edges e at v} G[e,v] J[r][e],
// G = +1 at the head (higher id), -1 at the tail; pull over the edge list of
// each vertex (vptr/vedge, sign in the low bit).
// --------------------------------------------------------------------------
__global__ void k_charge(int64_t nv, const int64_t* __restrict__ vptr, const int32_t* __restrict__ vedge,
                         const uint8_t* __restrict__ node_int, const double* __restrict__ J, int64_t ne,
                         double dt, double* __restrict__ q, int nrhs) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv * nrhs) return;
  int r = (int)(i / nv);
  int64_t v = i % nv;
  if (!node_int[v]) return;
  double s = 0.0;
  for (int64_t k = vptr[v]; k < vptr[v + 1]; ++k) {
    int32_t code = vedge[k];
    int32_t e = code >> 1;
    s += (code & 1 ? -1.0 : 1.0) * J[(int64_t)r * ne + e];
  }
  q[i] += dt * s;
}

// res[v] = (G^T (T e))_v + q_v with Te = T e given per unknown [nint][nrhs]
__global__ void k_gauss(int64_t nv, const int64_t* __restrict__ vptr, const int32_t* __restrict__ vedge,
                        const uint8_t* __restrict__ node_int, const int32_t* __restrict__ dof,
                        const double* __restrict__ Tx, const double* __restrict__ q, int nrhs,
                        double* __restrict__ res) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv * nrhs) return;
  int r = (int)(i / nv);
  int64_t v = i % nv;
  if (!node_int[v]) {
    res[i] = 0.0;
    return;
  }
  double s = 0.0;
  for (int64_t k = vptr[v]; k < vptr[v + 1]; ++k) {
    int32_t code = vedge[k];
    int32_t d = dof[code >> 1];
    if (d >= 0) s += (code & 1 ? -1.0 : 1.0) * Tx[(int64_t)d * nrhs + r];
  }
  res[i] = s + q[i];
}


// Per-step Gauss check (Sec. IV-B): the charge update q += dt G^T J^{n+1/2}
// and the maxima over vertices of |G^T (T e^{n+1}) + q| (interior vertices)
// and |q|.  Thread (v, r) = (t / nrhs, t % nrhs) of a workgroup of bs = 256 -
// 256 % nrhs threads (whole vertices, the right-hand sides of a vertex in
// neighbouring lanes: shared lists, contiguous J, Tx and q rows); the grid
// of kGaussBlocks workgroups strides over the vertices.  vdof lists the
// unknowns at each vertex (d << 1 | tail).  J and Tx are per unknown
// [nint][nrhs] (Tx nullptr: charge update only), q [nv][nrhs].  With part,
// the maxima of each workgroup go to part[blockIdx.x][2 r + {0, 1}] and
// k_gauss_max takes the maxima over workgroups (a NaN residual wins).
constexpr int kGaussBlocks = 1024;

__device__ __forceinline__ double nan_max(double a, double b) {
  return (a != a || b != b) ? NAN : fmax(a, b);
}

__global__ void __launch_bounds__(256) k_gauss_step(int64_t nv, int nrhs, const int64_t* __restrict__ vptr,
                                                    const int32_t* __restrict__ vdof,
                                                    const uint8_t* __restrict__ node_int,
                                                    const double* __restrict__ J, double dt,
                                                    const double* __restrict__ Tx, double* __restrict__ q,
                                                    double* __restrict__ part) {
  const int bs = 256 - 256 % nrhs, vpb = bs / nrhs;
  const int t = threadIdx.x, r = t % nrhs;
  double mres = 0.0, mq = 0.0;
  for (int64_t v = (int64_t)blockIdx.x * vpb + t / nrhs; t < bs && v < nv; v += (int64_t)gridDim.x * vpb) {
    if (!node_int[v]) continue;  // the charge of boundary vertices stays 0
    double sj = 0.0, st = 0.0;
    // batches of GB incident unknowns: their codes first, then all their
    // value loads in flight at once (reads past the list end are clamped
    // and not used), summed in list order
    constexpr int GB = 8;
    const int64_t k0 = vptr[v], k1 = vptr[v + 1];
    for (int64_t kb = k0; kb < k1; kb += GB) {
      int32_t code[GB];
#pragma unroll
      for (int u = 0; u < GB; ++u) code[u] = vdof[kb + u < k1 ? kb + u : k1 - 1];
      double jv[GB], tv[GB];
#pragma unroll
      for (int u = 0; u < GB; ++u) {
        const int64_t o = (int64_t)(code[u] >> 1) * nrhs + r;
        jv[u] = J[o];
        tv[u] = Tx ? Tx[o] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < GB; ++u)
        if (kb + u < k1) {
          const double sg = (code[u] & 1) ? -1.0 : 1.0;
          sj += sg * jv[u];
          st += sg * tv[u];
        }
    }
    const int64_t o = v * nrhs + r;
    const double qn = q[o] + dt * sj;
    q[o] = qn;
    mq = fmax(mq, fabs(qn));
    mres = nan_max(mres, fabs(st + qn));
  }
  if (!part) return;
  __shared__ double red[2][256];
  red[0][t] = mres;
  red[1][t] = mq;
  __syncthreads();
  if (t < nrhs) {
    double a = red[0][t], b = red[1][t];
    for (int u = t + nrhs; u < bs; u += nrhs) {
      a = nan_max(a, red[0][u]);
      b = fmax(b, red[1][u]);
    }
    part[(int64_t)blockIdx.x * 2 * kMaxRhs + 2 * t] = a;
    part[(int64_t)blockIdx.x * 2 * kMaxRhs + 2 * t + 1] = b;
  }
}

// Vector form of k_gauss_step: V right-hand sides per lane (nrhs a multiple
// of V; G = nrhs / V lanes per vertex), each gather one 8V-byte load.
template <int V>
__global__ void __launch_bounds__(256) k_gauss_step_v(int64_t nv, int nrhs, const int64_t* __restrict__ vptr,
                                                      const int32_t* __restrict__ vdof,
                                                      const uint8_t* __restrict__ node_int,
                                                      const double* __restrict__ J, double dt,
                                                      const double* __restrict__ Tx, double* __restrict__ q,
                                                      double* __restrict__ part) {
  const int G = nrhs / V;
  const int bs = 256 - 256 % G, vpb = bs / G;
  const int t = threadIdx.x, lq = t % G;
  double mres[V], mq[V];
#pragma unroll
  for (int w = 0; w < V; ++w) mres[w] = mq[w] = 0.0;
  for (int64_t v = (int64_t)blockIdx.x * vpb + t / G; t < bs && v < nv; v += (int64_t)gridDim.x * vpb) {
    if (!node_int[v]) continue;  // the charge of boundary vertices stays 0
    double sj[V], st[V];
#pragma unroll
    for (int w = 0; w < V; ++w) sj[w] = st[w] = 0.0;
    constexpr int GB = 8;
    const int64_t k0 = vptr[v], k1 = vptr[v + 1];
    for (int64_t kb = k0; kb < k1; kb += GB) {
      int32_t code[GB];
#pragma unroll
      for (int u = 0; u < GB; ++u) code[u] = vdof[kb + u < k1 ? kb + u : k1 - 1];
      double jv[GB][V], tv[GB][V];
#pragma unroll
      for (int u = 0; u < GB; ++u) {
        const int64_t o = (int64_t)(code[u] >> 1) * nrhs + lq * V;
        vload<double, V>(J + o, jv[u]);
        if (Tx) {
          vload<double, V>(Tx + o, tv[u]);
        } else {
#pragma unroll
          for (int w = 0; w < V; ++w) tv[u][w] = 0.0;
        }
      }
#pragma unroll
      for (int u = 0; u < GB; ++u)
        if (kb + u < k1) {
          const double sg = (code[u] & 1) ? -1.0 : 1.0;
#pragma unroll
          for (int w = 0; w < V; ++w) {
            sj[w] += sg * jv[u][w];
            st[w] += sg * tv[u][w];
          }
        }
    }
    const int64_t o = v * nrhs + lq * V;
    double qn[V];
    vload<double, V>(q + o, qn);
#pragma unroll
    for (int w = 0; w < V; ++w) {
      qn[w] = qn[w] + dt * sj[w];
      mq[w] = fmax(mq[w], fabs(qn[w]));
      mres[w] = nan_max(mres[w], fabs(st[w] + qn[w]));
    }
    vstore<double, V>(q + o, qn);
  }
  if (!part) return;
  __shared__ double red[2][256 * V];
#pragma unroll
  for (int w = 0; w < V; ++w) {
    red[0][t * V + w] = mres[w];
    red[1][t * V + w] = mq[w];
  }
  __syncthreads();
  if (t < nrhs) {
    const int g = t / V, w = t % V;
    double a = red[0][g * V + w], b = red[1][g * V + w];
    for (int u = g + G; u < bs; u += G) {
      a = nan_max(a, red[0][u * V + w]);
      b = fmax(b, red[1][u * V + w]);
    }
    part[(int64_t)blockIdx.x * 2 * kMaxRhs + 2 * t] = a;
    part[(int64_t)blockIdx.x * 2 * kMaxRhs + 2 * t + 1] = b;
  }
}

// out[2 r + {0, 1}] = the maxima of the nb workgroups' part rows: one
// workgroup of 1024 threads, value t = tid % 64 over the rows g, g + 16, ...
// of group g = tid / 64 (independent loads, eight in flight), then the 16
// group maxima through LDS (order-free: maxima)
__global__ void __launch_bounds__(1024) k_gauss_max(int nb, int nrhs, const double* __restrict__ part,
                                                    double* __restrict__ out) {
  __shared__ double gm[16][64];
  const int t = threadIdx.x & 63, g = threadIdx.x >> 6;
  const bool res = (t & 1) == 0;  // even values: residual maxima (NaN wins)
  double m = 0.0;
  if (t < 2 * nrhs) {
    for (int b0 = g; b0 < nb; b0 += 16 * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int b = b0 + 16 * u;
        v[u] = b < nb ? part[(int64_t)b * 2 * kMaxRhs + t] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) m = res ? nan_max(m, v[u]) : fmax(m, v[u]);
    }
  }
  gm[g][t] = m;
  __syncthreads();
  if (g == 0 && t < 2 * nrhs) {
    for (int k = 1; k < 16; ++k) m = res ? nan_max(m, gm[k][t]) : fmax(m, gm[k][t]);
    out[t] = m;
  }
}

// q [nv][nrhs] <- src [nrhs][nv] (or 0 with src == nullptr)
__global__ void k_charge_set(int64_t nv, int nrhs, const double* __restrict__ src, double* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv * nrhs) return;
  const int64_t v = i / nrhs;
  const int r = (int)(i % nrhs);
  q[i] = src ? src[(int64_t)r * nv + v] : 0.0;
}

// --------------------------------------------------------------------------
// Device-side bookkeeping of a captured refined step (FP32 factors, FP64
// refinement): the initial |b|^2, the relative residual after every solve,
// the gates that skip the sweeps no longer needed, and a snapshot of each
// solve's CG state, read back once after the step.
// --------------------------------------------------------------------------
constexpr int kMaxGraphSweeps = 4;
struct RefineState {
  double bn[kMaxRhs];                              // |b|^2 per RHS
  double gres[kMaxGraphSweeps + 1][kMaxRhs];       // |b - A x| / |b| after solves 0..S
  int gate[kMaxGraphSweeps + 2];                   // gate[k] = 1: sweep k (and all after) skipped
  int checked[kMaxGraphSweeps + 1];                // gres[k] was computed
  int ran[kMaxGraphSweeps + 1];                    // solve k ran
  int iters[kMaxGraphSweeps + 1][kMaxRhs];
  double rr[kMaxGraphSweeps + 1][kMaxRhs], rr0[kMaxGraphSweeps + 1][kMaxRhs];
  int done[kMaxGraphSweeps + 1], breakdown[kMaxGraphSweeps + 1];
};

// fixed-order sum of the kDotBlocks partials of rhs r ([kDotBlocks][kMaxRhs])
__device__ double partial_total(const double* __restrict__ pa, int nrhs, double* part) {
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

// clear the state; bn from the partials of b . b; gate[0] = 0
__global__ void __launch_bounds__(kScalarThreads) k_refine_init(int nrhs, const double* __restrict__ partial,
                                                                RefineState* __restrict__ rs) {
  __shared__ double part[kScalarThreads];
  int* w = reinterpret_cast<int*>(rs);
  for (size_t k = threadIdx.x; k < sizeof(RefineState) / sizeof(int); k += blockDim.x) w[k] = 0;
  __syncthreads();
  const double s = partial_total(partial, nrhs, part);
  if ((int)threadIdx.x < nrhs) rs->bn[threadIdx.x] = s;
}

// after solve k-1 (k >= 1): gres[k-1] = |r| / |b| from the partials of r . r,
// gate[k] = 1 when every RHS meets tol (the CG state is then marked done, so
// the gated solve's CG kernels return at once); a closed gate stays closed
__global__ void __launch_bounds__(kScalarThreads) k_refine_check(int k, int nrhs, const double* __restrict__ partial,
                                                                 double tol, RefineState* __restrict__ rs,
                                                                 CgState* __restrict__ cg) {
  __shared__ double part[kScalarThreads];
  __shared__ int all_ok;
  if (rs->gate[k - 1]) {
    if (threadIdx.x == 0) rs->gate[k] = 1;
    return;
  }
  if (threadIdx.x == 0) all_ok = 1;
  __syncthreads();
  const double s = partial_total(partial, nrhs, part);
  const int r = threadIdx.x;
  if (r < nrhs) {
    const double bn = rs->bn[r];
    const double g = bn > 0.0 ? sqrt(s / bn) : 0.0;
    rs->gres[k - 1][r] = g;
    if (!(g <= tol)) atomicAnd(&all_ok, 0);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    rs->checked[k - 1] = 1;
    rs->gate[k] = all_ok;
    if (all_ok) cg->done = 1;
  }
}

// snapshot of solve k's CG state (skipped with the solve)
__global__ void k_cg_snapshot(int k, int nrhs, const CgState* __restrict__ cg, RefineState* __restrict__ rs,
                              const int* __restrict__ gate) {
  if (gate && *gate) return;
  const int r = threadIdx.x;
  if (r < nrhs) {
    rs->iters[k][r] = cg->iters[r];
    rs->rr[k][r] = cg->rr[r];
    rs->rr0[k][r] = cg->rr0[r];
  }
  if (r == 0) {
    rs->ran[k] = 1;
    rs->done[k] = cg->done;
    rs->breakdown[k] = cg->breakdown;
  }
}

}  // namespace ddfem

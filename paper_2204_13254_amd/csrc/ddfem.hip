// Solver context and C ABI (include/ddfem.h).
//
// Per-step data flow of the decomposed solve (Sec. III-A, eq. (f1schur);
// local factors L_rr of [I | Gamma] with the corner rows L_cr and local
// corner Schur complements K_s).  Stored per subdomain (the local inverses
// of Sec. III-C, split by the factor's column blocks): Linv_II = L_II^-1;
// the couplings L_GI, L_cI as factored; Psi_G = L_cG L_GG^-1 in the corner
// rows; the interface block of the local inverse
// M = (K_rr^-1)_GG = L_GG^-T L_GG^-1.
//   pre-solve : w = owner split of b;  t_I = Linv_II w_I;
//               y_G = w_G - L_GI t_I;  g' = w_c - L_cI t_I;
//               z0 = K_cc^-1 sum_s B_c^T (g' - Psi_G y_G);
//               d = sum_s B_s (M y_G - Psi_G^T z0)
//   CG on F lambda = d with
//               F p = sum_s B_s (M v + Psi_G^T z_s),  v = B_s^T p,
//               z = K_cc^-1 sum_s B_c^T Psi_G v
//   recovery  : u = y_G - B_s^T lambda;
//               x_c = K_cc^-1 sum_s B_c^T (g' - Psi_G u);  x_G = M u - Psi_G^T x_c;
//               x_I = Linv_II^T (t_I - L_GI^T x_G - L_cI^T x_c);  e = owner's copy.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "ddfem.h"
#include "kernels.hpp"
#include "dp2.hpp"
#include "pic.hpp"
#include "mixed.hpp"
#include "plan.hpp"

namespace ddfem {

static thread_local std::string g_err;

struct DDError {
  int code;
  std::string msg;
};

#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      throw DDError{DD_ERR_HIP, std::string("HIP error ") + hipGetErrorString(e_) + " at " \
                                    + #x + " (line " + std::to_string(__LINE__) + ")"};   \
  } while (0)

static inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }
// grid of a kernel that maps workgroups to XCD-contiguous ranges (multiple of 8)
static inline unsigned nblk8(int64_t n) { return (nblk(n) + 7u) / 8u * 8u; }

template <class V>
static V* upload(const std::vector<V>& h, std::vector<void*>& owned, hipStream_t st) {
  V* d = nullptr;
  size_t bytes = std::max<size_t>(1, h.size()) * sizeof(V);
  hipError_t e = hipMalloc((void**)&d, bytes);
  if (e == hipErrorOutOfMemory) throw DDError{DD_ERR_OOM, "device allocation failed"};
  HIPCHK(e);
  owned.push_back(d);
  if (!h.empty()) {
    // the host vector may be freed right after: finish the copy here
    HIPCHK(hipMemcpyAsync(d, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  return d;
}

template <class V>
static V* dalloc(size_t n, std::vector<void*>& owned) {
  V* d = nullptr;
  hipError_t e = hipMalloc((void**)&d, std::max<size_t>(1, n) * sizeof(V));
  if (e == hipErrorOutOfMemory) throw DDError{DD_ERR_OOM, "device allocation failed"};
  HIPCHK(e);
  owned.push_back(d);
  return d;
}

struct Items {
  MvItem* d = nullptr;   // work items (one wave each), longest first
  int64_t n = 0;
  MvOut* outs = nullptr; // output blocks to reduce (split lists only)
  int64_t n_out = 0;
  int64_t n_slots = 0;   // partial slots used (0 = direct writes)
  int32_t* mlist = nullptr;  // tile list (ranges index it), or null for contiguous ranges
  void* partial = nullptr;   // own partial slots (lists that run beside others), or null
  bool pair = false;         // row-pair items (k_tile_mv2)
  bool oct = false;          // row-octet workgroup items (k_tile_mv8)
};

// Work-list shapes (longest tile range of one wave per product class, and
// the length buckets of the full passes).  Defaults measured on the 64^3
// box workload; dd_autotune picks them per context by timing candidates.
struct Tuning {
  int chunk = 32;         // interface-block and corner-row lists
  int coarse_chunk = 16;  // coarse lists: few and long (8: +10%, 4: +28% at 64^3)
  int full_chunk = 96;    // full r-block lists
  int full_bucket = 8;    // length buckets of the full lists' placement
  int full_persist = 0;   // full passes: workgroups of a persistent grid (0: one per work group)
  int full_pair = 0;      // full passes, 9..32 RHS: 1 = two output rows per wave sharing the input
                          // loads; 2 = eight rows per workgroup sharing them through LDS
  int full_quarter = 1;   // full passes: lanes of all-zero 16 x 16 tile quarters read the zero tile
  int sym_pw = 0;         // symmetric product: panel width (FP32: 2 or 4; 0 = 4; FP64: always 2)
  int sym_persist = 0;    // symmetric product: workgroups of a persistent grid (a multiple of 8), so
                          // that the corner and coarse chain beside it keeps free wave slots;
                          // 0 = one workgroup per four items
};

struct Ctx {
  Plan P;
  dd_options opt;
  int device = 0;  // current device at dd_setup (the stream's device)
  hipStream_t st = nullptr;
  // side stream: the interface-row products of an F application run there
  // while the coarse solve (a short chain of small launches) runs on st
  hipStream_t st2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // the factorisation's kernel sequence, captured once on two internal
  // streams (fa: subdomains, fb: coarse block) and replayed; ordered after
  // and before the caller's stream by ev_fa / ev_fb
  hipStream_t fa = nullptr, fb = nullptr;
  hipEvent_t ev_fa = nullptr, ev_fb = nullptr, ev_ffork = nullptr, ev_fjoin = nullptr;
  hipGraphExec_t factor_graph = nullptr;
  double dt = 0, beta = 0;
  int nrhs = 1;
  bool fp32 = false;
  bool factored = false;
  hipGraphExec_t cg_graph = nullptr;  // captured block of CG iterations
  int cg_graph_iters = 0;
  // captured refined solve of a step (pre-solve, CG, recovery, residual
  // checks and gated sweeps; FP32 factors with refinement, first variant):
  // CG iterations per solve and sweeps it holds, the last step's needs
  // (two of them, keyed by their buffers: the resident step alternates its
  // output slots)
  struct StepGraph {
    hipGraphExec_t g = nullptr;
    const double* b = nullptr;
    double *x = nullptr, *tx = nullptr, *sx = nullptr;
    int iters = 0, sweeps = 0;
    uint64_t used = 0;
  } step_graphs[2];
  uint64_t step_clock = 0;
  // resident Newmark state of dd_step_resident, unknown-major [nint][nrhs]:
  // slot rs_p holds e^n, the other e^{n-1}, each with its products T e and
  // S e; rs_j holds J^{n-1/2}.  rs_stale: the products predate the current
  // matrices (a new factorisation or permittivity).
  double *rs_e[2] = {nullptr, nullptr}, *rs_te[2] = {nullptr, nullptr}, *rs_se[2] = {nullptr, nullptr};
  double* rs_j = nullptr;
  int rs_p = 0;
  bool rs_alloc = false, rs_stale = false;
  int need_iters = 0, need_sweeps = 0;
  RefineState* d_rs = nullptr;
  RefineState* h_rs = nullptr;   // pinned
  double* d_rpart = nullptr;     // partial sums of the refinement norms [kDotBlocks][kMaxRhs]
  bool coarse_lists = false;  // coarse products use the nonzero-tile lists
  Tuning tuning;
  std::string tune_cache;     // dd_options.tune_cache, copied at setup ("" = none)
  bool tune_applied = false;  // dd_factor has run the tuner (or read its cache) once
  // output blocks of every product class (host), kept so that the work lists
  // can be rebuilt with other chunk lengths
  std::vector<MvItem> blk_corner_N, blk_corner_T, blk_co_N, blk_co_T, blk_full_N,
      blk_full_T, blk_cross_N, blk_cross_T;
  // per-row tile lists (host) of the I x I passes (L_II^-1) and of the
  // [Gamma; c] x I passes (L_GI, L_cI)
  std::vector<int32_t> ml_full_N, ml_full_T, ml_cross_N, ml_cross_T;
  void* d_zero_tile = nullptr;                // one zero tile (row-pair lists)
  std::vector<uint8_t> full_pattern;  // nonzero-tile flags the full lists were built from
  std::vector<void*> owned;

  // sizes
  int nsub = 0;  // subdomains; the coarse block is descriptor index nsub
  int Kc = 0;    // coarse tile rows
  int64_t ntiles = 0, rows_total = 0, coarse_row0 = 0;
  int max_kr = 0;
  std::vector<SubDev> subs_h;

  // device: mesh and elements
  double *d_coords = nullptr, *d_mu = nullptr, *d_eps = nullptr, *d_Te = nullptr, *d_Se = nullptr;
  int32_t* d_tsort = nullptr;
  SubDev* d_subs = nullptr;
  void* d_tiles = nullptr;   // factor store; operand-order tiles after dd_factor
  void* d_tilesT = nullptr;  // operand-order transposed tiles
  void* d_mtri = nullptr;    // interface blocks of the local inverses, packed lower, operand order
  int64_t* d_m_off = nullptr;   // first tile of each subdomain's block
  int64_t m_tiles = 0;
  void* d_partial_mv = nullptr;
  int64_t max_slots = 0;        // largest slot count of any work list
  int64_t partial_slots = 0;    // slots d_partial_mv holds
  void* d_scratch = nullptr;
  int64_t* d_scratch_off = nullptr;
  // per factor-store tile: L tile nonzero / inverse tile nonzero (every flag
  // a factorization reads it has written before)
  uint8_t* d_nzl = nullptr;
  uint8_t* d_nzi = nullptr;
  int* d_err = nullptr;
  // particle steps: per-tetrahedron geometry, face neighbours, edges, and
  // the counters of one launch (built on the first particle call)
  double* d_pic_geo = nullptr;
  int32_t *d_pic_nbr = nullptr, *d_pic_tedge = nullptr;
  unsigned long long* d_pic_cnt = nullptr;
  int32_t *d_pic_count = nullptr, *d_pic_bsum = nullptr;  // ordering by cell: [nt + 1], chunk totals
  // mixed E/B step (built on first use): canonical faces, their edges, the
  // faces of every tetrahedron, and the pull list unknown <- (tet, local edge)
  int64_t n_faces = 0;
  std::vector<int32_t> faces_h;  // [nf][3] vertices ascending
  int32_t *d_tet_faces = nullptr, *d_face_edges = nullptr, *d_e6list = nullptr;
  int64_t* d_e6ptr = nullptr;
  double* d_buf6 = nullptr;  // [nt][6][nrhs]
  double* d_bt = nullptr;    // face fluxes [nf][nrhs]
  // Robin dual-primal variant (method 1): one multiplier per side, in the
  // order of the interface rows (d_grow); R = 2 alpha M_T in side space
  double robin_alpha = 0.0;
  int32_t *d_code2 = nullptr, *d_partner2 = nullptr;
  int64_t* d_rrp = nullptr;
  double* d_rval = nullptr;
  int64_t n_radd = 0;            // Robin terms of the local interface blocks (lower triangle, no alpha)
  int64_t* d_radd_pos = nullptr;
  double* d_radd_val = nullptr;
  double *d_gmV = nullptr, *d_gm_rhs = nullptr, *d_lam2 = nullptr, *d_gm_partial = nullptr;
  double *d_gm_h = nullptr, *d_gm_tot = nullptr, *d_gm_y = nullptr, *d_gm_wpart = nullptr;
  double *d_gm_H = nullptr, *d_gm_cs = nullptr, *d_gm_sn = nullptr, *d_gm_g = nullptr;
  int64_t* d_rrow = nullptr;            // local row of every R column (side -> row)
  GmState* d_gm_st = nullptr;
  GmState* h_gm_st = nullptr;           // pinned copy of the GMRES state
  std::vector<hipGraphExec_t> gm_graphs;  // captured blocks of GMRES iterations
  // local assembly pull
  int64_t n_lent = 0;
  int64_t *d_lptr = nullptr, *d_ldest = nullptr;
  int32_t* d_lcon = nullptr;
  int64_t n_pad = 0;
  int64_t* d_padpos = nullptr;
  // coarse assembly pull
  int64_t n_cent = 0;
  int64_t *d_cptr = nullptr, *d_csrc = nullptr, *d_cdest = nullptr;
  // global CSR (T, S)
  int64_t nnz = 0;
  int64_t *d_rp = nullptr, *d_gptr = nullptr;
  int32_t *d_ci = nullptr, *d_gcon = nullptr;
  double2* d_vals = nullptr;
  // vector maps
  int32_t* d_rowsrc = nullptr;           // [rows_total]
  int64_t n_grow = 0;
  int64_t* d_grow = nullptr;             // interface-block rows
  int32_t* d_glam = nullptr;             // lambda code (id<<1 | negative) or -1
  int64_t *d_lrow0 = nullptr, *d_lrow1 = nullptr;
  int64_t *d_cgptr = nullptr, *d_cgrows = nullptr;  // coarse gather
  int64_t n_csc = 0;
  int64_t *d_cscrows = nullptr, *d_csccrow = nullptr;  // corner scatter
  int64_t* d_dsrc = nullptr;
  int32_t *d_interior = nullptr, *d_dof = nullptr, *d_tdof = nullptr;
  // Gauss law adjacency (interior edges only)
  int64_t* d_vptr = nullptr;
  int32_t* d_vedge = nullptr;
  uint8_t* d_nodeint = nullptr;
  double* d_vres = nullptr;  // [nv][nrhs] Gauss residual
  double* d_q = nullptr;     // accumulated nodal charge of the per-step check, [nv][nrhs]
  double* d_gmax = nullptr;   // maxima of the per-step check [nrhs][2]
  double* d_gpart = nullptr;  // their workgroup shares [kGaussBlocks][2 kMaxRhs]
  int32_t* d_vdof = nullptr; // vertex -> unknowns (d << 1 | tail), the lists of d_vedge
  // work lists
  // full_*: interior inverse factor L_II^-1; cross_*: the couplings L_GI,
  // L_cI of the interface and corner rows to the interior; co_*: coarse
  // inverse factor; corner_N / corner_T: Psi_Gamma u on the corner rows /
  // Psi_Gamma^T z onto the interface rows
  Items full_N, full_T, cross_N, cross_T, co_N, co_T, corner_N, corner_T;
  // symmetric product M u (panel pairs, partial slots, fixed-order reduce)
  struct SymList {
    SymItem* d = nullptr;
    int64_t n = 0;
    MvOut* outs = nullptr;
    int64_t n_out = 0;
    void* partial = nullptr;
    void* zero = nullptr;  // one zero tile (positions outside the stored triangle)
    int pw = 0;  // panel width the list was built for
  } sym;
  // work vectors
  void* X[10] = {};
  int64_t nlam = 0;
  double *d_d = nullptr, *d_lam = nullptr, *d_res = nullptr, *d_p = nullptr, *d_Fp = nullptr;
  // multipliers of the first solve of the last two steps (forward / adjoint),
  // for warm starts: previous value, or linear extrapolation 2 l^n - l^{n-1}
  struct Warm {
    double* cur = nullptr;
    double* old = nullptr;
    int have = 0;
  };
  Warm warm_fw, warm_adj;
  double* d_partial = nullptr;
  double* d_p2 = nullptr;  // p of odd CG iterations (even ones use d_p)
  double* d_z = nullptr;   // preconditioned residual
  double* d_partial2 = nullptr;  // second partial-sum array (r.r next to r.z)
  // lumped preconditioner K_lam (CSR in multiplier space) and its pull list
  int64_t lam_nnz = 0;
  int64_t *d_lrp = nullptr, *d_lgptr = nullptr;
  int32_t *d_lci = nullptr, *d_lgcon = nullptr;
  double* d_lvals = nullptr;
  CgState* d_cg = nullptr;
  CgState* h_cg = nullptr;  // pinned copy of the CG state
  double* h_partial = nullptr;  // pinned [kDotBlocks * kMaxRhs]
  // global vectors [nint][nrhs]
  double *g_b = nullptr, *g_e = nullptr, *g_r = nullptr, *g_x = nullptr, *g_t1 = nullptr, *g_t2 = nullptr,
         *g_t3 = nullptr, *g_t4 = nullptr;

  int64_t factor_bytes = 0, trailing_bytes = 0, schur_bytes = 0, corner_bytes = 0, coarse_bytes = 0,
          full_bytes = 0, cross_bytes = 0;

  // optional per-class kernel timing with HIP events on the solve stream
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_next = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  double prof_ms[DD_PROF_CLASSES] = {0};
  int64_t prof_n[DD_PROF_CLASSES] = {0};

  ~Ctx() {
    if (st) (void)hipStreamSynchronize(st);
    if (st2) (void)hipStreamSynchronize(st2);
    if (fa) (void)hipStreamSynchronize(fa);
    if (fb) (void)hipStreamSynchronize(fb);
    if (factor_graph) (void)hipGraphExecDestroy(factor_graph);
    for (hipEvent_t e : {ev_fa, ev_fb, ev_ffork, ev_fjoin})
      if (e) (void)hipEventDestroy(e);
    if (fa) (void)hipStreamDestroy(fa);
    if (fb) (void)hipStreamDestroy(fb);
    if (cg_graph) (void)hipGraphExecDestroy(cg_graph);
    for (auto& sg : step_graphs)
      if (sg.g) (void)hipGraphExecDestroy(sg.g);
    for (hipGraphExec_t g : gm_graphs)
      if (g) (void)hipGraphExecDestroy(g);
    if (h_gm_st) (void)hipHostFree(h_gm_st);
    if (h_rs) (void)hipHostFree(h_rs);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (st2) (void)hipStreamDestroy(st2);
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (void* p : owned) (void)hipFree(p);
    if (h_cg) (void)hipHostFree(h_cg);
    if (h_partial) (void)hipHostFree(h_partial);
  }
};

// ---------------------------------------------------------------------------
// setup
// ---------------------------------------------------------------------------
// Work list of one batched product.  Every output block whose tile range is
// longer than kChunkTiles is split into chunks writing partial slots, then
// summed by k_mv_reduce.
//
// Placement: workgroups are dispatched round-robin over the 8 XCDs (group b
// runs on XCD b % 8) and each XCD has its own L2.  All items of one
// subdomain read the same input blocks, so subdomains are assigned to XCDs
// (greedy by tile count) and the list is interleaved so that group b only
// holds items of XCD b % 8, longest first (measured on par with a single
// global longest-first list; placing each subdomain's items consecutively
// was slightly slower).  With bucket > 1 the lengths are compared in
// buckets and the given order is kept inside a bucket: the full passes hand
// in neighbouring rows of a subdomain next to each other, so the four waves
// of a workgroup read the same input blocks at about the same time (1.525 ->
// 1.497 ms per full pass at 64^3 with buckets of 8; 4: 1.505, 16: 1.496).
// Padding items (s = -1) fill the ragged end.
constexpr int kXcds = 8;
constexpr int kWavesPerGroup = 4;

template <class It, class SubF, class LenF>
static std::vector<It> place_xcd(int nsub, const std::vector<It>& v, const It& pad, SubF sub, LenF len,
                                 int bucket = 1, int per_group = kWavesPerGroup) {
  // XCD assignment: subdomains by greedy load; the coarse block (a single
  // "subdomain" holding many items, with small shared inputs) round-robin
  std::vector<int64_t> load_s(nsub + 1, 0);
  for (const It& it : v) load_s[sub(it)] += len(it) + 1;
  std::vector<int32_t> order(nsub);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return load_s[a] > load_s[b]; });
  std::vector<int> xcd_of(nsub + 1, 0);
  int64_t xload[kXcds] = {0};
  for (int s : order) {
    int best = 0;
    for (int x = 1; x < kXcds; ++x)
      if (xload[x] < xload[best]) best = x;
    xcd_of[s] = best;
    xload[best] += load_s[s];
  }
  std::vector<std::vector<It>> lists(kXcds);
  int rr = 0;
  for (const It& it : v) {
    int x = sub(it) < nsub ? xcd_of[sub(it)] : (rr++ % kXcds);
    lists[x].push_back(it);
  }
  size_t groups = 0;
  // within an XCD: longest first
  for (auto& L : lists) {
    std::stable_sort(L.begin(), L.end(), [&](const It& a, const It& b) { return len(a) / bucket > len(b) / bucket; });
    groups = std::max(groups, (L.size() + per_group - 1) / per_group);
  }
  std::vector<It> placed(groups * kXcds * per_group, pad);
  for (size_t g = 0; g < groups; ++g)
    for (int x = 0; x < kXcds; ++x)
      for (int w = 0; w < per_group; ++w) {
        size_t k = g * per_group + w;
        if (k < lists[x].size()) placed[(g * kXcds + x) * per_group + w] = lists[x][k];
      }
  if (v.empty()) placed.clear();
  return placed;
}

static Items make_items(Ctx& C, const std::vector<MvItem>& blocks, int chunk, bool grouped = false, int bucket = 1) {
  bool split = false;
  for (const MvItem& b : blocks)
    if (b.hi - b.lo > chunk) split = true;
  std::vector<MvItem> v;
  std::vector<int32_t> chunk_of;
  std::vector<MvOut> outs;
  int32_t slot = 0;
  for (const MvItem& b : blocks) {
    if (!split) {
      v.push_back({b.s, b.o, b.lo, b.hi, -1, 0, b.o2, -1});
      chunk_of.push_back(0);
      continue;
    }
    int32_t n = std::max(1, (b.hi - b.lo + chunk - 1) / chunk);
    if (n == 1) {
      // a row that fits one wave writes its output directly (no partial)
      v.push_back({b.s, b.o, b.lo, b.hi, -1, 0, b.o2, -1});
      chunk_of.push_back(0);
      continue;
    }
    // n partial slots per output block (2n for a row pair: o's, then o2's)
    int32_t oidx = (int32_t)outs.size();
    outs.push_back({b.s, b.o, slot, n});
    if (b.o2 >= 0) outs.push_back({b.s, b.o2, slot + n, n});
    for (int32_t c = 0; c < n; ++c) {
      int32_t lo = b.lo + c * chunk, hi = std::min(b.hi, lo + chunk);
      v.push_back({b.s, b.o, lo, std::max(lo, hi), slot + c, oidx, b.o2, b.o2 >= 0 ? slot + n + c : -1});
      chunk_of.push_back(c);
    }
    slot += b.o2 >= 0 ? 2 * n : n;
  }
  if (grouped && split) {
    // chunk-major inside a subdomain, so that neighbouring rows (similar
    // tile lists, the same input blocks) sit in one workgroup
    std::vector<int32_t> ord(v.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
      if (v[a].s != v[b].s) return v[a].s < v[b].s;
      return chunk_of[a] < chunk_of[b];
    });
    std::vector<MvItem> w(v.size());
    for (size_t k = 0; k < ord.size(); ++k) w[k] = v[ord[k]];
    v.swap(w);
  }
  std::vector<MvItem> placed = place_xcd(
      C.nsub, v, MvItem{-1, 0, 0, 0, -1, 0}, [](const MvItem& a) { return a.s; },
      [](const MvItem& a) { return (int64_t)(a.hi - a.lo); }, grouped ? bucket : 1);
  Items it;
  it.n = (int64_t)placed.size();
  it.d = upload(placed, C.owned, C.st);
  it.n_slots = slot;
  if (split) {
    it.n_out = (int64_t)outs.size();
    it.outs = upload(outs, C.owned, C.st);
  }
  C.max_slots = std::max<int64_t>(C.max_slots, slot);
  return it;
}

// panel width of the symmetric product (accumulators per wave: 2 PW blocks)
template <class T>
constexpr int sym_panel() {
  return sizeof(T) == 4 ? 4 : 2;
}

static void release(Ctx& C, void* p);

// panel width of the symmetric product for the context's precision and tuning
static int sym_width(const Ctx& C) {
  if (!C.fp32) return sym_panel<double>();
  return C.tuning.sym_pw == 2 ? 2 : sym_panel<float>();
}

// Work list of the symmetric product: panel pairs (P, Q), P >= Q, of every
// subdomain's interface tiles; kG * nP partial slots per subdomain.  A
// previous list (another panel width) is released.
static void make_sym_list(Ctx& C, int pw, size_t wsz) {
  release(C, C.sym.d);
  release(C, C.sym.outs);
  release(C, C.sym.partial);
  release(C, C.sym.zero);
  C.sym = Ctx::SymList{};
  C.sym.pw = pw;
  std::vector<SymItem> v;
  std::vector<MvOut> outs;
  int64_t slot = 0;
  for (int s = 0; s < C.nsub; ++s) {
    const SubDev& q = C.subs_h[s];
    if (q.kG == 0) continue;
    const int nP = (q.kG + pw - 1) / pw;
    for (int P = 0; P < nP; ++P)
      for (int Q = 0; Q <= P; ++Q) v.push_back({s, P, Q, (int32_t)slot});
    for (int b = 0; b < q.kG; ++b) outs.push_back({s, q.kI + b, (int32_t)(slot + (int64_t)b * nP), nP});
    slot += (int64_t)q.kG * nP;
    if (slot >= INT32_MAX) throw DDError{DD_ERR_OOM, "too many partial slots"};
  }
  std::vector<SymItem> placed = place_xcd(
      C.nsub, v, SymItem{-1, 0, 0, 0}, [](const SymItem& a) { return a.s; },
      [&](const SymItem& a) { return (int64_t)(a.P == a.Q ? pw * (pw + 1) / 2 : pw * pw); });
  C.sym.n = (int64_t)placed.size();
  C.sym.d = upload(placed, C.owned, C.st);
  C.sym.n_out = (int64_t)outs.size();
  C.sym.outs = upload(outs, C.owned, C.st);
  void* p = nullptr;
  HIPCHK(hipMalloc(&p, std::max<int64_t>(1, slot) * kTile * C.nrhs * wsz / NB));
  C.owned.push_back(p);
  C.sym.partial = p;
  HIPCHK(hipMalloc(&p, kTile * wsz));
  C.owned.push_back(p);
  HIPCHK(hipMemsetAsync(p, 0, kTile * wsz, C.st));
  C.sym.zero = p;
}

static void build_device(Ctx& C, const double* coords) {
  Plan& P = C.P;
  hipStream_t st = C.st;
  const int nsub = P.nsub;
  C.nsub = nsub;
  const int64_t nc = P.ncorner();
  C.Kc = (int)((nc + NB - 1) / NB);
  // ---- descriptors --------------------------------------------------------
  C.subs_h.resize(nsub + 1);
  int64_t toff = 0, roff = 0;
  C.max_kr = 0;
  for (int s = 0; s <= nsub; ++s) {
    SubDev q{};
    if (s < nsub) {
      const SubInfo& si = P.subs[s];
      q.nI = si.nI; q.nG = si.nG; q.nC = si.nC;
      q.kI = si.kI; q.kG = si.kG; q.kC = si.kC; q.K = si.K;
      C.max_kr = std::max(C.max_kr, si.kr());
    } else {
      q.nI = (int32_t)nc; q.nG = 0; q.nC = 0;
      q.kI = C.Kc; q.kG = 0; q.kC = 0; q.K = C.Kc;
      C.coarse_row0 = roff;
    }
    q.tile_off = toff;
    q.row_off = roff;
    toff += (int64_t)q.K * (q.K + 1) / 2;
    roff += (int64_t)q.K * NB;
    C.subs_h[s] = q;
    if (s < nsub) {
      P.subs[s].tile_off = q.tile_off;
      P.subs[s].row_off = q.row_off;
    }
  }
  C.ntiles = toff;
  C.rows_total = roff;
  const size_t wsz = C.fp32 ? 4 : 8;
  for (const SubDev& q : C.subs_h)
    if (q.K - 1 > kColList)
      throw DDError{DD_ERR_OOM, "a factor block has more than " + std::to_string(kColList + 1) + " tile rows"};
  C.d_subs = upload(C.subs_h, C.owned, st);
  {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<int64_t>(1, C.ntiles) * kTile * wsz);
    if (e == hipErrorOutOfMemory) throw DDError{DD_ERR_OOM, "device allocation of the factor store failed"};
    HIPCHK(e);
    C.owned.push_back(p);
    C.d_tiles = p;
    p = nullptr;
    e = hipMalloc(&p, std::max<int64_t>(1, C.ntiles) * kTile * wsz);
    if (e == hipErrorOutOfMemory) throw DDError{DD_ERR_OOM, "device allocation of the transposed store failed"};
    HIPCHK(e);
    C.owned.push_back(p);
    C.d_tilesT = p;
    C.d_nzl = dalloc<uint8_t>(std::max<int64_t>(1, C.ntiles), C.owned);
    C.d_nzi = dalloc<uint8_t>(std::max<int64_t>(1, C.ntiles), C.owned);
    std::vector<int64_t> mo(nsub);
    int64_t acc = 0;
    for (int s = 0; s < nsub; ++s) {
      mo[s] = acc;
      acc += (int64_t)C.subs_h[s].kG * (C.subs_h[s].kG + 1) / 2;
    }
    C.m_tiles = acc;
    C.d_m_off = upload(mo, C.owned, st);
    p = nullptr;
    e = hipMalloc(&p, std::max<int64_t>(1, C.m_tiles) * kTile * wsz);
    if (e == hipErrorOutOfMemory) throw DDError{DD_ERR_OOM, "device allocation of the interface inverse failed"};
    HIPCHK(e);
    C.owned.push_back(p);
    C.d_mtri = p;
  }
  // algorithmic byte counts (unpadded, packed triangles)
  C.factor_bytes = (2 * C.ntiles + C.m_tiles) * kTile * (int64_t)wsz;
  for (int s = 0; s < nsub; ++s) {
    const SubInfo& q = P.subs[s];
    int64_t nr = q.nI + q.nG;
    // inverse-factor triangle plus the premultiplied corner rows it carries
    C.trailing_bytes += ((int64_t)q.nG * (q.nG + 1) / 2 + (int64_t)q.nC * q.nG) * wsz;
    C.schur_bytes += (int64_t)q.nG * (q.nG + 1) / 2 * wsz;
    C.corner_bytes += (int64_t)q.nC * q.nG * wsz;
    // (before the nonzero-tile lists exist: dense I x I and [Gamma; c] x I)
    C.full_bytes += ((int64_t)q.nI * (q.nI + 1) / 2) * wsz;
    C.cross_bytes += ((int64_t)(q.nG + q.nC) * q.nI) * wsz;
    (void)nr;
  }
  C.coarse_bytes = nc * (nc + 1) / 2 * (int64_t)wsz;
  // scratch rows for the triangular inversion
  {
    std::vector<int64_t> so(nsub + 1);
    int64_t acc = 0;
    for (int s = 0; s <= nsub; ++s) {
      so[s] = acc;
      acc += C.subs_h[s].kI + C.subs_h[s].kG;
    }
    C.d_scratch_off = upload(so, C.owned, st);
    void* p = nullptr;
    HIPCHK(hipMalloc(&p, std::max<int64_t>(1, acc) * kTile * wsz));
    C.owned.push_back(p);
    C.d_scratch = p;
  }
  C.d_err = dalloc<int>(1, C.owned);

  // ---- mesh arrays ------------------------------------------------------------
  std::vector<double> ch(coords, coords + 3 * P.nv);
  C.d_coords = upload(ch, C.owned, st);
  C.d_tsort = upload(P.tsort, C.owned, st);
  C.d_mu = dalloc<double>(P.nt, C.owned);
  C.d_eps = dalloc<double>(P.nt, C.owned);
  C.d_Te = dalloc<double>(P.nt * 36, C.owned);
  C.d_Se = dalloc<double>(P.nt * 36, C.owned);

  // ---- local assembly pull lists -------------------------------------------------
  std::vector<std::vector<int64_t>> tets_of(nsub);
  for (int64_t t = 0; t < P.nt; ++t) tets_of[P.part[t]].push_back(t);
  std::vector<int32_t> dof2row(P.nint, -1);
  std::vector<int64_t> lptr{0}, ldest;
  std::vector<int32_t> lcon;
  std::vector<int64_t> padpos;
  std::vector<std::pair<int64_t, int32_t>> pairs;
  for (int s = 0; s < nsub; ++s) {
    const SubInfo& q = P.subs[s];
    const SubDev& qd = C.subs_h[s];
    const auto& L = P.local[s];
    for (int32_t p = 0; p < (int32_t)L.size(); ++p) dof2row[L[p]] = P.padded_row(s, p);
    pairs.clear();
    for (int64_t t : tets_of[s])
      for (int a = 0; a < 6; ++a) {
        int32_t da = P.dof[P.tet_edges[t * 6 + a]];
        if (da < 0) continue;
        for (int b = 0; b < 6; ++b) {
          int32_t db = P.dof[P.tet_edges[t * 6 + b]];
          if (db < 0) continue;
          int32_t ra = dof2row[da], rb = dof2row[db];
          if (ra < rb) continue;
          int64_t ti = qd.tile_off + (int64_t)(ra / NB) * (ra / NB + 1) / 2 + rb / NB;
          int64_t pos = ti * kTile + (ra % NB) * NB + (rb % NB);
          pairs.emplace_back(pos, (int32_t)(t * 36 + a * 6 + b));
        }
      }
    std::sort(pairs.begin(), pairs.end());
    for (size_t i = 0; i < pairs.size();) {
      size_t j = i;
      while (j < pairs.size() && pairs[j].first == pairs[i].first) {
        lcon.push_back(pairs[j].second);
        ++j;
      }
      ldest.push_back(pairs[i].first);
      lptr.push_back((int64_t)lcon.size());
      i = j;
    }
    for (int32_t p : L) dof2row[p] = -1;
    // padding diagonals
    auto add_pad = [&](int32_t r0, int32_t r1) {
      for (int32_t r = r0; r < r1; ++r) {
        int64_t ti = qd.tile_off + (int64_t)(r / NB) * (r / NB + 1) / 2 + r / NB;
        padpos.push_back(ti * kTile + (r % NB) * NB + (r % NB));
      }
    };
    add_pad(q.nI, q.kI * NB);
    add_pad(q.kI * NB + q.nG, q.kr() * NB);
    add_pad(q.kr() * NB + q.nC, q.K * NB);
  }
  {
    const SubDev& qc = C.subs_h[nsub];
    for (int32_t r = (int32_t)nc; r < C.Kc * NB; ++r) {
      int64_t ti = qc.tile_off + (int64_t)(r / NB) * (r / NB + 1) / 2 + r / NB;
      padpos.push_back(ti * kTile + (r % NB) * NB + (r % NB));
    }
  }
  C.n_lent = (int64_t)ldest.size();
  C.d_lptr = upload(lptr, C.owned, st);
  C.d_ldest = upload(ldest, C.owned, st);
  C.d_lcon = upload(lcon, C.owned, st);
  C.n_pad = (int64_t)padpos.size();
  C.d_padpos = upload(padpos, C.owned, st);
  std::vector<int64_t>().swap(lptr);
  std::vector<int64_t>().swap(ldest);
  std::vector<int32_t>().swap(lcon);

  // ---- coarse assembly pull lists --------------------------------------------------
  {
    std::vector<std::pair<int64_t, int64_t>> cp;
    const SubDev& qc = C.subs_h[nsub];
    for (int s = 0; s < nsub; ++s) {
      const SubInfo& q = P.subs[s];
      const SubDev& qd = C.subs_h[s];
      const auto& L = P.local[s];
      int32_t base = q.nI + q.nG;
      int32_t r0 = q.kr() * NB;
      for (int32_t a = 0; a < q.nC; ++a) {
        int32_t I = P.dof_corner[L[base + a]];
        for (int32_t b = 0; b < q.nC; ++b) {
          int32_t J = P.dof_corner[L[base + b]];
          if (I < J) continue;
          int32_t ra = r0 + a, rb = r0 + b;
          if (ra < rb) std::swap(ra, rb);
          int64_t sti = qd.tile_off + (int64_t)(ra / NB) * (ra / NB + 1) / 2 + rb / NB;
          int64_t spos = sti * kTile + (ra % NB) * NB + (rb % NB);
          int64_t dti = qc.tile_off + (int64_t)(I / NB) * (I / NB + 1) / 2 + J / NB;
          int64_t dpos = dti * kTile + (I % NB) * NB + (J % NB);
          cp.emplace_back(dpos, spos);
        }
      }
    }
    std::sort(cp.begin(), cp.end());
    std::vector<int64_t> cptr{0}, csrc, cdest;
    for (size_t i = 0; i < cp.size();) {
      size_t j = i;
      while (j < cp.size() && cp[j].first == cp[i].first) csrc.push_back(cp[j++].second);
      cdest.push_back(cp[i].first);
      cptr.push_back((int64_t)csrc.size());
      i = j;
    }
    C.n_cent = (int64_t)cdest.size();
    C.d_cptr = upload(cptr, C.owned, st);
    C.d_csrc = upload(csrc, C.owned, st);
    C.d_cdest = upload(cdest, C.owned, st);
  }

  // ---- global CSR pattern of (T, S) and its pull list ------------------------------
  {
    std::vector<std::pair<uint64_t, int32_t>> gp;
    gp.reserve(P.nt * 36);
    for (int64_t t = 0; t < P.nt; ++t)
      for (int a = 0; a < 6; ++a) {
        int32_t da = P.dof[P.tet_edges[t * 6 + a]];
        if (da < 0) continue;
        for (int b = 0; b < 6; ++b) {
          int32_t db = P.dof[P.tet_edges[t * 6 + b]];
          if (db < 0) continue;
          gp.emplace_back((uint64_t)da * (uint64_t)P.nint + (uint64_t)db, (int32_t)(t * 36 + a * 6 + b));
        }
      }
    std::sort(gp.begin(), gp.end());
    std::vector<int64_t> rp(P.nint + 1, 0), gptr{0};
    std::vector<int32_t> ci, gcon;
    gcon.reserve(gp.size());
    for (size_t i = 0; i < gp.size();) {
      size_t j = i;
      while (j < gp.size() && gp[j].first == gp[i].first) gcon.push_back(gp[j++].second);
      uint64_t key = gp[i].first;
      int64_t row = (int64_t)(key / (uint64_t)P.nint);
      ci.push_back((int32_t)(key % (uint64_t)P.nint));
      rp[row + 1]++;
      gptr.push_back((int64_t)gcon.size());
      i = j;
    }
    for (int64_t r = 0; r < P.nint; ++r) rp[r + 1] += rp[r];
    C.nnz = (int64_t)ci.size();
    C.d_rp = upload(rp, C.owned, st);
    C.d_ci = upload(ci, C.owned, st);
    C.d_gptr = upload(gptr, C.owned, st);
    C.d_gcon = upload(gcon, C.owned, st);
    C.d_vals = dalloc<double2>(C.nnz, C.owned);
  }

  // ---- vector maps -------------------------------------------------------------------
  {
    std::vector<int32_t> rowsrc(C.rows_total, -1);
    std::vector<int64_t> grow;
    std::vector<int32_t> glam;
    std::vector<int64_t> cscrows, csccrow;
    // lambda id per (subdomain, unpadded position) for interface rows
    std::vector<std::vector<int32_t>> lam_at(nsub);
    for (int s = 0; s < nsub; ++s) lam_at[s].assign(P.subs[s].nG, -1);
    for (int64_t l = 0; l < P.nlambda(); ++l) {
      int s0 = P.lam_s0[l], s1 = P.lam_s1[l];
      lam_at[s0][P.lam_p0[l] - P.subs[s0].nI] = (int32_t)(l << 1);
      lam_at[s1][P.lam_p1[l] - P.subs[s1].nI] = (int32_t)((l << 1) | 1);
    }
    for (int s = 0; s < nsub; ++s) {
      const SubInfo& q = P.subs[s];
      const SubDev& qd = C.subs_h[s];
      const auto& L = P.local[s];
      for (int32_t p = 0; p < (int32_t)L.size(); ++p) {
        int32_t d = L[p];
        if (P.owner[d] == s) rowsrc[qd.row_off + P.padded_row(s, p)] = d;
      }
      for (int32_t r = q.kI * NB; r < q.kr() * NB; ++r) {
        grow.push_back(qd.row_off + r);
        int32_t g = r - q.kI * NB;
        glam.push_back(g < q.nG ? lam_at[s][g] : -1);
      }
      for (int32_t r = q.kr() * NB; r < q.K * NB; ++r) {
        int32_t c = r - q.kr() * NB;
        cscrows.push_back(qd.row_off + r);
        csccrow.push_back(c < q.nC ? C.coarse_row0 + P.dof_corner[L[q.nI + q.nG + c]] : -1);
      }
    }
    C.d_rowsrc = upload(rowsrc, C.owned, st);
    C.n_grow = (int64_t)grow.size();
    C.d_grow = upload(grow, C.owned, st);
    C.d_glam = upload(glam, C.owned, st);
    C.n_csc = (int64_t)cscrows.size();
    C.d_cscrows = upload(cscrows, C.owned, st);
    C.d_csccrow = upload(csccrow, C.owned, st);
    // multipliers
    C.nlam = P.nlambda();
    std::vector<int64_t> r0(C.nlam), r1(C.nlam);
    for (int64_t l = 0; l < C.nlam; ++l) {
      r0[l] = C.subs_h[P.lam_s0[l]].row_off + P.padded_row(P.lam_s0[l], P.lam_p0[l]);
      r1[l] = C.subs_h[P.lam_s1[l]].row_off + P.padded_row(P.lam_s1[l], P.lam_p1[l]);
    }
    C.d_lrow0 = upload(r0, C.owned, st);
    C.d_lrow1 = upload(r1, C.owned, st);
    // pattern and pull list of the lumped preconditioner K_lam: the tets of
    // subdomain s couple the multipliers of its interface edges, with the
    // signs of B_s (+ in the lower subdomain id)
    {
      if (P.nt > INT32_MAX / 72) throw DDError{DD_ERR_ARG, "too many tetrahedra for the preconditioner pull list"};
      std::vector<int32_t> dlam(P.nint, -1);
      for (int64_t l = 0; l < C.nlam; ++l) dlam[P.lam_dof[l]] = (int32_t)l;
      std::vector<std::pair<uint64_t, int32_t>> kp;
      for (int64_t t = 0; t < P.nt; ++t) {
        const int32_t sub = P.part[t];
        for (int a = 0; a < 6; ++a) {
          const int32_t da = P.dof[P.tet_edges[t * 6 + a]];
          const int32_t la = da >= 0 ? dlam[da] : -1;
          if (la < 0) continue;
          const bool na = P.lam_s0[la] != sub;
          for (int b = 0; b < 6; ++b) {
            const int32_t db = P.dof[P.tet_edges[t * 6 + b]];
            const int32_t lb = db >= 0 ? dlam[db] : -1;
            if (lb < 0) continue;
            const bool nb = P.lam_s0[lb] != sub;
            kp.emplace_back((uint64_t)la * (uint64_t)C.nlam + (uint64_t)lb,
                            (int32_t)(((t * 36 + a * 6 + b) << 1) | (na != nb ? 1 : 0)));
          }
        }
      }
      std::sort(kp.begin(), kp.end());
      std::vector<int64_t> lrp(C.nlam + 1, 0), lgptr{0};
      std::vector<int32_t> lci, lgcon;
      lgcon.reserve(kp.size());
      for (size_t i = 0; i < kp.size();) {
        size_t j = i;
        while (j < kp.size() && kp[j].first == kp[i].first) lgcon.push_back(kp[j++].second);
        lrp[(int64_t)(kp[i].first / (uint64_t)C.nlam) + 1]++;
        lci.push_back((int32_t)(kp[i].first % (uint64_t)C.nlam));
        lgptr.push_back((int64_t)lgcon.size());
        i = j;
      }
      for (int64_t l = 0; l < C.nlam; ++l) lrp[l + 1] += lrp[l];
      C.lam_nnz = (int64_t)lci.size();
      C.d_lrp = upload(lrp, C.owned, st);
      C.d_lci = upload(lci, C.owned, st);
      C.d_lgptr = upload(lgptr, C.owned, st);
      C.d_lgcon = upload(lgcon, C.owned, st);
      C.d_lvals = dalloc<double>(C.lam_nnz, C.owned);
    }
    // coarse gather: corner c <- its subdomain corner rows, ascending subdomain
    std::vector<int64_t> cgptr((int64_t)C.Kc * NB + 1, 0), cgrows;
    std::vector<std::vector<int64_t>> byc(nc);
    for (int s = 0; s < nsub; ++s) {
      const SubInfo& q = P.subs[s];
      const auto& L = P.local[s];
      for (int32_t c = 0; c < q.nC; ++c)
        byc[P.dof_corner[L[q.nI + q.nG + c]]].push_back(C.subs_h[s].row_off + q.kr() * NB + c);
    }
    for (int64_t c = 0; c < (int64_t)C.Kc * NB; ++c) {
      if (c < nc)
        for (int64_t r : byc[c]) cgrows.push_back(r);
      cgptr[c + 1] = (int64_t)cgrows.size();
    }
    C.d_cgptr = upload(cgptr, C.owned, st);
    C.d_cgrows = upload(cgrows, C.owned, st);
    // owner's copy of each unknown
    std::vector<int64_t> dsrc(P.nint);
    for (int s = 0; s < nsub; ++s) {
      const auto& L = P.local[s];
      for (int32_t p = 0; p < (int32_t)L.size(); ++p) {
        int32_t d = L[p];
        if (P.owner[d] != s) continue;
        dsrc[d] = P.dof_corner[d] >= 0 ? C.coarse_row0 + P.dof_corner[d]
                                       : C.subs_h[s].row_off + P.padded_row(s, p);
      }
    }
    C.d_dsrc = upload(dsrc, C.owned, st);
    C.d_interior = upload(P.interior, C.owned, st);
    C.d_dof = upload(P.dof, C.owned, st);
    std::vector<int32_t> tdof(P.nt * 6);
    for (int64_t i = 0; i < P.nt * 6; ++i) tdof[i] = P.dof[P.tet_edges[i]];
    C.d_tdof = upload(tdof, C.owned, st);
  }
  // ---- Gauss-law adjacency: interior edges at each vertex ------------------------
  {
    std::vector<int64_t> vptr(P.nv + 1, 0);
    for (int64_t d = 0; d < P.nint; ++d) {
      int32_t e = P.interior[d];
      vptr[P.edges[2 * e] + 1]++;
      vptr[P.edges[2 * e + 1] + 1]++;
    }
    for (int64_t v = 0; v < P.nv; ++v) vptr[v + 1] += vptr[v];
    std::vector<int32_t> vedge(vptr[P.nv]);
    std::vector<int64_t> fill(vptr.begin(), vptr.end() - 1);
    for (int64_t d = 0; d < P.nint; ++d) {
      int32_t e = P.interior[d];
      vedge[fill[P.edges[2 * e + 1]]++] = e << 1;        // head: +1
      vedge[fill[P.edges[2 * e]]++] = (e << 1) | 1;      // tail: -1
    }
    C.d_vptr = upload(vptr, C.owned, st);
    C.d_vedge = upload(vedge, C.owned, st);
    C.d_nodeint = upload(P.node_interior, C.owned, st);
    C.d_vres = dalloc<double>(P.nv * C.nrhs, C.owned);
    C.d_q = dalloc<double>(P.nv * C.nrhs, C.owned);
    HIPCHK(hipMemsetAsync(C.d_q, 0, P.nv * C.nrhs * sizeof(double), st));
    C.d_gmax = dalloc<double>((size_t)kMaxRhs * 2, C.owned);
    C.d_gpart = dalloc<double>((size_t)kGaussBlocks * kMaxRhs * 2, C.owned);
    std::vector<int32_t> vdof(vedge.size());
    for (size_t k = 0; k < vedge.size(); ++k) vdof[k] = (P.dof[vedge[k] >> 1] << 1) | (vedge[k] & 1);
    C.d_vdof = upload(vdof, C.owned, st);
  }
  // ---- work lists --------------------------------------------------------------------
  {
    // corner rows Psi_Gamma u over the interface columns, and Psi_Gamma^T z
    // onto the interface rows of subdomains with corners; coarse inverse
    // factor rows (the r-block lists are built from the nonzero tiles after
    // the first factorisation)
    std::vector<MvItem> oN, oT, cN, cT;
    for (int s = 0; s < nsub; ++s) {
      const SubDev& q = C.subs_h[s];
      const int kr = q.kI + q.kG;
      for (int o = kr; o < q.K; ++o) cN.push_back({s, o, q.kI, kr, -1, 0});
      if (q.kC > 0)
        for (int o = q.kI; o < kr; ++o) cT.push_back({s, o, kr, q.K, -1, 0});
    }
    for (int o = 0; o < C.Kc; ++o) {
      oN.push_back({nsub, o, 0, o + 1, -1, 0});
      oT.push_back({nsub, o, o, C.Kc, -1, 0});
    }
    // runs beside the coarse chain: own partial slots
    make_sym_list(C, sym_width(C), wsz);
    C.corner_N = make_items(C, cN, C.tuning.chunk);
    // (summing the symmetric partials inside this pass instead of a reduce on
    // the side stream measured slower: it lengthens the main-stream chain)
    C.corner_T = make_items(C, cT, C.tuning.chunk);
    C.co_N = make_items(C, oN, C.tuning.chunk);
    C.co_T = make_items(C, oT, C.tuning.chunk);
    C.blk_corner_N.swap(cN);
    C.blk_corner_T.swap(cT);
    void* p = nullptr;
    HIPCHK(hipMalloc(&p, std::max<int64_t>(1, C.max_slots) * kTile * C.nrhs * wsz / NB));
    C.owned.push_back(p);
    C.d_partial_mv = p;
    C.partial_slots = std::max<int64_t>(1, C.max_slots);
  }
  // ---- work vectors --------------------------------------------------------------------
  const int nr = C.nrhs;
  for (int i = 0; i < 10; ++i) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<int64_t>(1, C.rows_total) * nr * wsz);
    if (e == hipErrorOutOfMemory) throw DDError{DD_ERR_OOM, "device allocation failed"};
    HIPCHK(e);
    C.owned.push_back(p);
    C.X[i] = p;
    HIPCHK(hipMemsetAsync(p, 0, std::max<int64_t>(1, C.rows_total) * nr * wsz, st));
  }
  const int64_t nl = std::max<int64_t>(1, C.nlam) * nr;
  C.d_d = dalloc<double>(nl, C.owned);
  C.d_lam = dalloc<double>(nl, C.owned);
  C.d_res = dalloc<double>(nl, C.owned);
  C.d_p = dalloc<double>(nl, C.owned);
  C.d_Fp = dalloc<double>(nl, C.owned);
  C.warm_fw.cur = dalloc<double>(nl, C.owned);
  C.warm_fw.old = dalloc<double>(nl, C.owned);
  C.warm_adj.cur = dalloc<double>(nl, C.owned);
  C.warm_adj.old = dalloc<double>(nl, C.owned);
  C.d_partial = dalloc<double>(kDotBlocks * kMaxRhs, C.owned);
  C.d_p2 = dalloc<double>(nl, C.owned);
  C.d_z = dalloc<double>(nl, C.owned);
  C.d_partial2 = dalloc<double>(kDotBlocks * kMaxRhs, C.owned);
  C.d_cg = dalloc<CgState>(1, C.owned);
  HIPCHK(hipHostMalloc((void**)&C.h_cg, sizeof(CgState), hipHostMallocDefault));
  HIPCHK(hipHostMalloc((void**)&C.h_partial, sizeof(double) * kDotBlocks * kMaxRhs, hipHostMallocDefault));
  C.d_rs = dalloc<RefineState>(1, C.owned);
  HIPCHK(hipHostMalloc((void**)&C.h_rs, sizeof(RefineState), hipHostMallocDefault));
  C.d_rpart = dalloc<double>((size_t)kDotBlocks * kMaxRhs, C.owned);
  const int64_t ng = std::max<int64_t>(1, P.nint) * nr;
  C.g_b = dalloc<double>(ng, C.owned);
  C.g_e = dalloc<double>(ng, C.owned);
  C.g_r = dalloc<double>(ng, C.owned);
  C.g_x = dalloc<double>(ng, C.owned);
  C.g_t1 = dalloc<double>(ng, C.owned);
  C.g_t2 = dalloc<double>(ng, C.owned);
  C.g_t3 = dalloc<double>(ng, C.owned);
  C.g_t4 = dalloc<double>(ng, C.owned);
  HIPCHK(hipStreamSynchronize(st));
}

// Drop the captured graphs (they hold work lists, buffers and iteration
// counts that are about to change); the next solve captures them again.
static void drop_graphs(Ctx& C) {
  if (C.cg_graph) HIPCHK(hipGraphExecDestroy(C.cg_graph));
  C.cg_graph = nullptr;
  for (auto& sg : C.step_graphs) {
    if (sg.g) HIPCHK(hipGraphExecDestroy(sg.g));
    sg = Ctx::StepGraph{};
  }
  for (hipGraphExec_t& g : C.gm_graphs) {
    if (g) HIPCHK(hipGraphExecDestroy(g));
    g = nullptr;
  }
}

// ---------------------------------------------------------------------------
// factor
// ---------------------------------------------------------------------------
// dynamic LDS of a tile-chain kernel: the list of up to n term indices
static inline unsigned chain_lds(int n) { return (unsigned)(std::max(n, 2) * sizeof(uint16_t) + 15) & ~15u; }

// Blocked Cholesky of the [I|Gamma] rows of blocks s0 .. s0+cnt-1 (corner
// rows get L_cr and the Schur complement K_s = A_cc - L_cr L_cr^T).
template <class T>
static void factor_chol(Ctx& C, int s0, int cnt, hipStream_t st) {
  T* tiles = (T*)C.d_tiles;
  int max_kr = 0;
  for (int s = s0; s < s0 + cnt; ++s)
    max_kr = std::max(max_kr, C.subs_h[s].kI + C.subs_h[s].kG);
  for (int k = 0; k < max_kr; ++k) {
    int tmax = 0;
    for (int s = s0; s < s0 + cnt; ++s) {
      const SubDev& q = C.subs_h[s];
      if (k < q.kI + q.kG) tmax = std::max(tmax, q.K - k - 1);
    }
    hipLaunchKernelGGL(k_potrf<T>, dim3(cnt), dim3(256), 0, st, k, s0, tiles, C.d_subs, C.d_err,
                       C.d_nzl, C.d_nzi);
    if (tmax > 0) {
      hipLaunchKernelGGL(k_trsm<T>, dim3(tmax, cnt), dim3(256), 0, st, k, s0, tiles, C.d_subs, C.d_nzl);
      // pairs of nonzero column tiles, strided over at most 64K workgroups
      // (2048 for one block: its nonzero pairs per step are a few thousand)
      const int64_t np = (int64_t)tmax * (tmax + 1) / 2;
      const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>({np, 65536 / cnt, 2048}));
      hipLaunchKernelGGL(k_syrk<T>, dim3(gx, cnt), dim3(256), 0, st, k, s0, tiles, C.d_subs,
                         (const uint8_t*)C.d_nzl);
    }
  }
  HIPCHK(hipGetLastError());
}

// Inverse factor Linv_rr row by row, then Psi = L_cr Linv_rr.
template <class T>
static void factor_inv(Ctx& C, int s0, int cnt, hipStream_t st) {
  T* tiles = (T*)C.d_tiles;
  int max_kr = 0;
  for (int s = s0; s < s0 + cnt; ++s)
    max_kr = std::max(max_kr, C.subs_h[s].kI + C.subs_h[s].kG);
  for (int i = 1; i < max_kr; ++i) {
    hipLaunchKernelGGL(k_trtri_row<T>, dim3(i, cnt), dim3(256), chain_lds(i), st, i, s0, (const T*)tiles, C.d_subs,
                       C.d_scratch_off, (T*)C.d_scratch, (const uint8_t*)C.d_nzl, C.d_nzi);
    hipLaunchKernelGGL(k_trtri_copy<T>, dim3(i, cnt), dim3(256), 0, st, i, s0, tiles, C.d_subs,
                       C.d_scratch_off, (const T*)C.d_scratch);
  }
  int max_kc = 0;
  for (int s = s0; s < s0 + cnt; ++s) max_kc = std::max(max_kc, C.subs_h[s].kC);
  for (int c = 0; c < max_kc && max_kr > 0; ++c) {
    hipLaunchKernelGGL(k_psi_row<T>, dim3(max_kr, cnt), dim3(256), chain_lds(max_kr), st, c, s0, (const T*)tiles, C.d_subs,
                       C.d_scratch_off, (T*)C.d_scratch, (const uint8_t*)C.d_nzl, (const uint8_t*)C.d_nzi);
    hipLaunchKernelGGL(k_psi_copy<T>, dim3(max_kr, cnt), dim3(256), 0, st, c, s0, tiles, C.d_subs,
                       C.d_scratch_off, (const T*)C.d_scratch);
  }
  HIPCHK(hipGetLastError());
}

// nonzero count of every tile in [t0, t0 + n) of the factor store
template <class T>
// (and, with qmask, the nonzero 16 x 16 quarters of every tile, operand order)
static std::vector<int32_t> tile_nnz(Ctx& C, int64_t t0, int64_t n, std::vector<int32_t>* qmask = nullptr) {
  std::vector<int32_t> nnz(n);
  if (qmask) qmask->assign(n, 0);
  if (n == 0) return nnz;
  int32_t* d_nnz = nullptr;
  HIPCHK(hipMalloc((void**)&d_nnz, 2 * n * sizeof(int32_t)));
  hipLaunchKernelGGL(k_tile_nnz<T>, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, C.st, t0, n, (const T*)C.d_tiles, d_nnz,
                     qmask ? d_nnz + n : (int32_t*)nullptr);
  HIPCHK(hipMemcpyAsync(nnz.data(), d_nnz, n * sizeof(int32_t), hipMemcpyDeviceToHost, C.st));
  if (qmask)
    HIPCHK(hipMemcpyAsync(qmask->data(), d_nnz + n, n * sizeof(int32_t), hipMemcpyDeviceToHost, C.st));
  HIPCHK(hipStreamSynchronize(C.st));
  HIPCHK(hipFree(d_nnz));
  return nnz;
}

static void release(Ctx& C, void* p) {
  if (!p) return;
  auto it = std::find(C.owned.begin(), C.owned.end(), p);
  if (it != C.owned.end()) C.owned.erase(it);
  HIPCHK(hipFree(p));
}

static void release_items(Ctx& C, Items& it) {
  release(C, it.d);
  release(C, it.outs);
  release(C, it.mlist);
  it = Items{};
}

// Split lists with short chunks may need more partial slots than were
// allocated.  The old buffer stays allocated: a captured graph may use it.
template <class T>
static void ensure_partial(Ctx& C) {
  if (C.max_slots <= C.partial_slots) return;
  void* p = nullptr;
  HIPCHK(hipMalloc(&p, C.max_slots * kNB * C.nrhs * sizeof(T)));
  C.owned.push_back(p);
  C.d_partial_mv = p;
  C.partial_slots = C.max_slots;
}

// Replace the coarse work lists by lists of the nonzero tiles of the coarse
// inverse factor (fixed by the corner order, so built once).
template <class T>
static void coarse_tile_lists(Ctx& C) {
  const SubDev& qc = C.subs_h[C.nsub];
  const int K = qc.K;
  const int64_t nt = (int64_t)K * (K + 1) / 2;
  std::vector<int32_t> nnz = tile_nnz<T>(C, qc.tile_off, nt);
  auto at = [&](int i, int j) { return nnz[(int64_t)i * (i + 1) / 2 + j]; };
  std::vector<int32_t> ln, lt;
  std::vector<MvItem> bn, bt;
  int64_t entries = 0;
  for (int o = 0; o < K; ++o) {
    int32_t b = (int32_t)ln.size();
    for (int j = 0; j <= o; ++j)
      if (at(o, j)) {
        ln.push_back(j);
        entries += at(o, j);
      }
    bn.push_back({C.nsub, o, b, (int32_t)ln.size(), -1, 0});
    b = (int32_t)lt.size();
    for (int i = o; i < K; ++i)
      if (at(i, o)) lt.push_back(i);
    bt.push_back({C.nsub, o, b, (int32_t)lt.size(), -1, 0});
  }
  // few output blocks: short chunks so that the product fills the device
  release_items(C, C.co_N);
  release_items(C, C.co_T);
  C.co_N = make_items(C, bn, C.tuning.coarse_chunk);
  C.co_N.mlist = upload(ln, C.owned, C.st);
  C.co_T = make_items(C, bt, C.tuning.coarse_chunk);
  C.co_T.mlist = upload(lt, C.owned, C.st);
  C.blk_co_N.swap(bn);
  C.blk_co_T.swap(bt);
  C.coarse_bytes = entries * (int64_t)sizeof(T);
  C.coarse_lists = true;
  ensure_partial<T>(C);
}

// Work items of the full passes from the per-row tile lists, single rows or
// row pairs (C.tuning.full_pair, 9..32 RHS): rows 2k and 2k+1 of a subdomain
// walk the union of their lists, flagged per entry (kPairMask).  At 64^3
// 96-tile chunks keep every single row in one wave (48 tiles: 1.465 ms per
// pass, 64: 1.444, 80: 1.432, 96: 1.430, 128: 1.432).
template <class T>
static void build_full_items(Ctx& C) {
  release_items(C, C.full_N);
  release_items(C, C.full_T);
  release_items(C, C.cross_N);
  release_items(C, C.cross_T);
  const bool pair = C.tuning.full_pair && C.nrhs > 8;
  const bool oct = pair && C.tuning.full_pair == 2;
  auto make_oct = [&](const std::vector<MvItem>& blk, const std::vector<int32_t>& ml, Items& it) {
    std::vector<int32_t> ol;
    std::vector<MvItem> ob;
    for (size_t k = 0; k < blk.size();) {
      size_t n = 1;
      while (n < 8 && k + n < blk.size() && blk[k + n].s == blk[k].s) ++n;
      std::vector<int32_t> pos(n);
      for (size_t j = 0; j < n; ++j) pos[j] = blk[k + j].lo;
      const int32_t b0 = (int32_t)ol.size();
      for (;;) {  // merge of n ascending lists, one flag bit per row
        int32_t m = INT32_MAX;
        for (size_t j = 0; j < n; ++j)
          if (pos[j] < blk[k + j].hi) m = std::min(m, ml[pos[j]] & kListMask);
        if (m == INT32_MAX) break;
        int32_t e = m;
        for (size_t j = 0; j < n; ++j)
          if (pos[j] < blk[k + j].hi && (ml[pos[j]] & kListMask) == m) {
            e |= 1 << (23 + j);
            ++pos[j];
          }
        ol.push_back(e);
      }
      ob.push_back({blk[k].s, blk[k].o, b0, (int32_t)ol.size(), -1, 0, (int32_t)n, -1});
      k += n;
    }
    std::vector<MvItem> placed = place_xcd(
        C.nsub, ob, MvItem{-1, 0, 0, 0, -1, 0}, [](const MvItem& a) { return a.s; },
        [](const MvItem& a) { return (int64_t)(a.hi - a.lo); }, C.tuning.full_bucket, 1);
    it.n = (int64_t)placed.size();
    it.d = upload(placed, C.owned, C.st);
    it.mlist = upload(ol, C.owned, C.st);
    it.oct = true;
  };
  auto make = [&](const std::vector<MvItem>& blk, const std::vector<int32_t>& ml_all, Items& it) {
    // zero-quarter flags only when the tuning asks for them
    std::vector<int32_t> stripped;
    if (!C.tuning.full_quarter) {
      stripped.resize(ml_all.size());
      for (size_t k = 0; k < ml_all.size(); ++k) stripped[k] = ml_all[k] & kListMask;
    }
    const std::vector<int32_t>& ml = C.tuning.full_quarter ? ml_all : stripped;
    if (oct) {
      make_oct(blk, ml, it);
      return;
    }
    if (!pair) {
      it = make_items(C, blk, C.tuning.full_chunk, true, C.tuning.full_bucket);
      it.mlist = upload(ml, C.owned, C.st);
      return;
    }
    std::vector<int32_t> pl;
    std::vector<MvItem> pb;
    for (size_t k = 0; k < blk.size(); ++k) {
      const MvItem& a = blk[k];
      const bool has2 = k + 1 < blk.size() && blk[k + 1].s == a.s;
      const int32_t b0 = (int32_t)pl.size();
      // single-row entry m | zero quarters << 25 -> pair entry fields
      auto mm = [&](int32_t e) { return e & kListMask; };
      auto qz = [&](int32_t e) { return (e >> 25) & 15; };
      if (!has2) {
        for (int32_t e = a.lo; e < a.hi; ++e) pl.push_back(mm(ml[e]) | qz(ml[e]) << 21 | (1 << 29));
        pb.push_back({a.s, a.o, b0, (int32_t)pl.size(), -1, 0});
        continue;
      }
      const MvItem& b = blk[k + 1];
      int32_t i = a.lo, j = b.lo;
      while (i < a.hi || j < b.hi) {  // merge of two ascending lists
        const int32_t ma = i < a.hi ? mm(ml[i]) : INT32_MAX, mb = j < b.hi ? mm(ml[j]) : INT32_MAX;
        const int32_t m = std::min(ma, mb);
        int32_t e = m;
        if (ma == m) e |= qz(ml[i]) << 21 | (1 << 29);
        if (mb == m) e |= qz(ml[j]) << 25 | (1 << 30);
        pl.push_back(e);
        if (ma == m) ++i;
        if (mb == m) ++j;
      }
      pb.push_back({a.s, a.o, b0, (int32_t)pl.size(), -1, 0, b.o, -1});
      ++k;
    }
    it = make_items(C, pb, C.tuning.full_chunk, true, C.tuning.full_bucket);
    it.mlist = upload(pl, C.owned, C.st);
    it.pair = true;
  };
  if (!C.d_zero_tile) {
    C.d_zero_tile = dalloc<T>(kTile, C.owned);
    HIPCHK(hipMemsetAsync(C.d_zero_tile, 0, kTile * sizeof(T), C.st));
  }
  make(C.blk_full_N, C.ml_full_N, C.full_N);
  make(C.blk_full_T, C.ml_full_T, C.full_T);
  make(C.blk_cross_N, C.ml_cross_N, C.cross_N);
  make(C.blk_cross_T, C.ml_cross_T, C.cross_T);
  ensure_partial<T>(C);
}

// Lists of the nonzero tiles of the r-block columns of I for the forward /
// transposed passes: the I x I block (L_II^-1, "full") and the [Gamma; c] x I
// block (L_GI and L_cI, "cross").  The interior nested-dissection order
// leaves whole tiles of L_II^-1 zero, and L_GI, L_cI keep the factor's
// sparsity.  The pattern is checked after every factorisation and the lists
// rebuilt when it changed, so a tile is skipped only while it is exactly zero.
template <class T>
static void full_tile_lists(Ctx& C) {
  const int64_t nt = C.subs_h[C.nsub].tile_off;  // subdomain tiles come first
  std::vector<int32_t> qm;
  std::vector<int32_t> nnz = tile_nnz<T>(C, 0, nt, &qm);
  std::vector<uint8_t> pat(nt);
  for (int64_t t = 0; t < nt; ++t) pat[t] = (uint8_t)(nnz[t] != 0 ? 16 | qm[t] : 0);
  if (pat == C.full_pattern && C.full_N.d) return;
  // zero quarters of a listed tile, in the layout of the store read: the
  // transposed store swaps the off-diagonal quarters
  auto zq = [&](int64_t t, bool transposed) -> int32_t {
    int32_t z = ~qm[t] & 15;
    if (transposed) z = (z & 9) | ((z & 2) << 1) | ((z & 4) >> 1);
    return z;
  };
  std::vector<int32_t> ln, lt, xn, xt;
  std::vector<MvItem> bn, bt, cn, ct;
  int64_t entries = 0, xentries = 0;
  for (int s = 0; s < C.nsub; ++s) {
    const SubDev& q = C.subs_h[s];
    const int kI = q.kI;
    auto tid = [&](int i, int j) { return q.tile_off + (int64_t)i * (i + 1) / 2 + j; };
    auto at = [&](int i, int j) { return nnz[tid(i, j)]; };
    if (q.K >= kPairMask) throw DDError{DD_ERR_OOM, "too many tile rows in a subdomain"};
    if (kI == 0) continue;
    // forward: I rows over I columns; [Gamma; c] rows over I columns
    for (int o = 0; o < q.K; ++o) {
      const bool irow = o < kI;
      std::vector<int32_t>& L = irow ? ln : xn;
      int32_t b = (int32_t)L.size();
      for (int j = 0; j <= std::min(o, kI - 1); ++j)
        if (at(o, j)) {
          L.push_back(j | zq(tid(o, j), false) << 25);
          (irow ? entries : xentries) += at(o, j);
        }
      (irow ? bn : cn).push_back({s, o, b, (int32_t)L.size(), -1, 0});
    }
    // transposed: I outputs over the I rows, and over the [Gamma; c] rows
    for (int o = 0; o < kI; ++o) {
      int32_t b = (int32_t)lt.size();
      for (int i = o; i < kI; ++i)
        if (at(i, o)) lt.push_back(i | zq(tid(i, o), true) << 25);
      bt.push_back({s, o, b, (int32_t)lt.size(), -1, 0});
      b = (int32_t)xt.size();
      for (int i = kI; i < q.K; ++i)
        if (at(i, o)) xt.push_back(i | zq(tid(i, o), true) << 25);
      ct.push_back({s, o, b, (int32_t)xt.size(), -1, 0});
    }
  }
  for (const auto* v : {&ln, &lt, &xn, &xt})
    if ((int64_t)v->size() >= INT32_MAX) throw DDError{DD_ERR_OOM, "tile lists exceed 2^31 entries"};
  C.blk_full_N.swap(bn);
  C.blk_full_T.swap(bt);
  C.ml_full_N.swap(ln);
  C.ml_full_T.swap(lt);
  C.blk_cross_N.swap(cn);
  C.blk_cross_T.swap(ct);
  C.ml_cross_N.swap(xn);
  C.ml_cross_T.swap(xt);
  C.full_bytes = entries * (int64_t)sizeof(T);
  C.cross_bytes = xentries * (int64_t)sizeof(T);
  C.full_pattern.swap(pat);
  build_full_items<T>(C);
}

template <class T>
static void autotune(Ctx& C, const char* cache, dd_tuning* out);

// The factorisation's kernels (element matrices, local assembly, blocked
// Cholesky, inverse factors, coarse block on the side stream, packing), in
// launch order on st and side; captured once per context and replayed.
template <class T>
static void factor_sequence(Ctx& C, hipStream_t st, hipStream_t side) {
  Plan& P = C.P;
  T* tiles = (T*)C.d_tiles;
  // (fills by kernel: the sequence is captured into a graph)
  {
    const int64_t n16 = std::max<int64_t>(1, C.ntiles) * kTile * (int64_t)sizeof(T) / 16;
    hipLaunchKernelGGL(k_clear16, dim3((unsigned)std::min<int64_t>(nblk(n16), 65536)), dim3(256), 0, st, n16,
                       (uint4*)tiles);
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, st, C.d_err, (int)INT32_MAX);
  }
  hipLaunchKernelGGL(k_element, dim3(nblk(P.nt)), dim3(256), 0, st, (int64_t)P.nt, C.d_coords, C.d_tsort,
                     C.d_mu, C.d_Te, C.d_Se);
  hipLaunchKernelGGL(k_pull_local<T>, dim3(nblk(C.n_lent)), dim3(256), 0, st, C.n_lent, C.d_lptr, C.d_lcon,
                     C.d_ldest, C.d_Te, C.d_Se, C.d_eps, C.beta * C.dt * C.dt, tiles);
  if (C.n_pad)
    hipLaunchKernelGGL(k_pad_diag<T>, dim3(nblk(C.n_pad)), dim3(256), 0, st, C.n_pad, C.d_padpos, tiles);
  if (C.n_radd)
    hipLaunchKernelGGL(k_add_entries<T>, dim3(nblk(C.n_radd)), dim3(256), 0, st, C.n_radd, C.d_radd_pos,
                       C.d_radd_val, C.robin_alpha, tiles);
  hipLaunchKernelGGL(k_pull_csr, dim3(nblk(C.nnz)), dim3(256), 0, st, C.nnz, C.d_gptr, C.d_gcon, C.d_Te,
                     C.d_Se, C.d_eps, C.d_vals);
  if (C.lam_nnz)
    hipLaunchKernelGGL(k_pull_lam, dim3(nblk(C.lam_nnz)), dim3(256), 0, st, C.lam_nnz, C.d_lgptr, C.d_lgcon,
                       C.d_Te, C.d_Se, C.d_eps, C.beta * C.dt * C.dt, C.d_lvals);
  HIPCHK(hipGetLastError());
  factor_chol<T>(C, 0, C.nsub, st);
  // The coarse matrix needs only the subdomains' Schur corner blocks: its
  // assembly and factorisation (a chain of small launches) run on the side
  // stream while the subdomains' inverse factors are formed on st.  The two
  // touch disjoint tiles (corner blocks are read; r rows, corner rows of the
  // r columns and the coarse block are written) and disjoint scratch rows.
  if (C.Kc > 0) HIPCHK(hipEventRecord(C.ev_ffork, st));
  factor_inv<T>(C, 0, C.nsub, st);
  {
    int max_kg = 0;
    for (int s = 0; s < C.nsub; ++s) max_kg = std::max(max_kg, C.subs_h[s].kG);
    if (max_kg > 0)
      hipLaunchKernelGGL(k_schur_inv<T>, dim3((unsigned)(max_kg * (max_kg + 1) / 2), C.nsub), dim3(256),
                         chain_lds(max_kg), st, 0,
                         (const T*)tiles, C.d_subs, C.d_m_off, (T*)C.d_mtri, (const uint8_t*)C.d_nzi);
  }
  if (C.Kc > 0) {
    HIPCHK(hipStreamWaitEvent(side, C.ev_ffork, 0));
    if (C.n_cent)
      hipLaunchKernelGGL(k_pull_coarse<T>, dim3(nblk(C.n_cent)), dim3(256), 0, side, C.n_cent, C.d_cptr,
                         C.d_csrc, C.d_cdest, tiles);
    factor_chol<T>(C, C.nsub, 1, side);
    factor_inv<T>(C, C.nsub, 1, side);
    HIPCHK(hipEventRecord(C.ev_fjoin, side));
    HIPCHK(hipStreamWaitEvent(st, C.ev_fjoin, 0));
  }
  if (C.ntiles > 0)
    hipLaunchKernelGGL(k_pack_tiles<T>, dim3((unsigned)C.ntiles), dim3(256), 0, st, C.ntiles, tiles,
                       (T*)C.d_tilesT);
  HIPCHK(hipGetLastError());
}

template <class T>
static int factor_impl(Ctx& C) {
  hipStream_t st = C.st;
  // the work lists may change with the factor's nonzero pattern: captured
  // solves are dropped, and the next step runs eagerly to size its capture
  HIPCHK(hipStreamSynchronize(st));
  drop_graphs(C);
  C.need_iters = C.need_sweeps = 0;
  HIPCHK(hipEventRecord(C.ev_fa, st));
  HIPCHK(hipStreamWaitEvent(C.fa, C.ev_fa, 0));
  if (!C.factor_graph) {
    HIPCHK(hipStreamBeginCapture(C.fa, hipStreamCaptureModeThreadLocal));
    hipGraph_t g = nullptr;
    try {
      factor_sequence<T>(C, C.fa, C.fb);
    } catch (...) {
      (void)hipStreamEndCapture(C.fa, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIPCHK(hipStreamEndCapture(C.fa, &g));
    HIPCHK(hipGraphInstantiate(&C.factor_graph, g, nullptr, nullptr, 0));
    HIPCHK(hipGraphDestroy(g));
  }
  HIPCHK(hipGraphLaunch(C.factor_graph, C.fa));
  HIPCHK(hipEventRecord(C.ev_fb, C.fa));
  HIPCHK(hipStreamWaitEvent(st, C.ev_fb, 0));
  HIPCHK(hipGetLastError());
  if (C.Kc > 0 && !C.coarse_lists) coarse_tile_lists<T>(C);
  full_tile_lists<T>(C);
  int err = 0;
  HIPCHK(hipMemcpyAsync(&err, C.d_err, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (err != INT32_MAX) {
    C.factored = false;
    if (err == C.nsub) throw DDError{DD_ERR_NOT_SPD, "coarse corner matrix is not positive definite"};
    throw DDError{DD_ERR_NOT_SPD, "non-positive or non-finite pivot in subdomain " + std::to_string(err)};
  }
  C.factored = true;
  C.warm_fw.have = C.warm_adj.have = 0;
  C.rs_stale = C.rs_alloc;  // the resident state's products predate these matrices
  if (!C.tune_cache.empty() && !C.tune_applied) autotune<T>(C, C.tune_cache.c_str(), nullptr);
  return DD_OK;
}

// ---------------------------------------------------------------------------
// solve
// ---------------------------------------------------------------------------
static void prof_resolve(Ctx& C) {
  if (C.ev_pending.empty()) return;
  HIPCHK(hipStreamSynchronize(C.st));
  for (auto& p : C.ev_pending) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, p.second.first, p.second.second));
    C.prof_ms[p.first] += ms;
    C.prof_n[p.first] += 1;
  }
  C.ev_pending.clear();
  C.ev_next = 0;
}

// record_start = false: the caller attaches both events to its launch
static bool prof_begin(Ctx& C, int cls, hipEvent_t* a, hipEvent_t* b, bool record_start = true) {
  if (!C.prof) return false;
  if (C.ev_next + 2 > C.ev_pool.size()) prof_resolve(C);
  while (C.ev_pool.size() < C.ev_next + 2) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    C.ev_pool.push_back(e);
  }
  *a = C.ev_pool[C.ev_next++];
  *b = C.ev_pool[C.ev_next++];
  C.ev_pending.push_back({cls, {*a, *b}});
  if (record_start) HIPCHK(hipEventRecord(*a, C.st));
  return true;
}

static int item_class(const Ctx& C, const Items& it) {
  if (&it == &C.corner_N || &it == &C.corner_T) return DD_PROF_CORNER;
  if (&it == &C.full_N || &it == &C.full_T) return DD_PROF_FULL;
  if (&it == &C.cross_N || &it == &C.cross_T) return DD_PROF_CROSS;
  return DD_PROF_COARSE;
}

template <class T, int NV, int NB16, int CLS, int LD>
static void mv_launch(Ctx& C, hipStream_t s, const Items& it, bool trans, const void* in, void* out, const void* add,
                      T alpha, const void* add_c, T alpha_c, const int* skip) {
  const bool split = it.n_out > 0;
  const T* tiles = (const T*)(trans ? C.d_tilesT : C.d_tiles);
  T* partial = (T*)(it.partial ? it.partial : C.d_partial_mv);
  // work groups come in multiples of 8 (one per XCD); a persistent grid is
  // a multiple of 8 too, so each workgroup stays on its groups' XCD
  int64_t grid = (it.n + 3) / 4;
  if ((CLS == DD_PROF_FULL || CLS == DD_PROF_CROSS) && C.tuning.full_persist > 0)
    grid = std::min<int64_t>(grid, C.tuning.full_persist);
  if constexpr (NV == 0) {
    if (it.oct) {
      int64_t g8 = it.n;  // one workgroup per item (a multiple of 8)
      if (C.tuning.full_persist > 0) g8 = std::min<int64_t>(g8, C.tuning.full_persist);
      hipLaunchKernelGGL((k_tile_mv8<T, NB16, CLS, LD>), dim3((unsigned)g8), dim3(256), 0, s, it.n, it.d, C.d_subs,
                         tiles, (const T*)in, (T*)out, (const T*)add, alpha, (const T*)add_c, alpha_c, C.nrhs,
                         (int)trans, (const int32_t*)it.mlist, skip, (const T*)C.d_zero_tile);
    } else if (it.pair) {
      hipLaunchKernelGGL((k_tile_mv2<T, NB16, CLS, LD>), dim3((unsigned)grid), dim3(256), 0, s, it.n, it.d, C.d_subs,
                         tiles, (const T*)in, (T*)out, (const T*)add, alpha, (const T*)add_c, alpha_c, C.nrhs,
                         (int)trans, partial, (const int32_t*)it.mlist, skip, (const T*)C.d_zero_tile);
    } else {
      hipLaunchKernelGGL((k_tile_mv<T, NV, NB16, CLS, LD>), dim3((unsigned)grid), dim3(256), 0, s, it.n, it.d,
                         C.d_subs, tiles, (const T*)in, (T*)out, (const T*)add, alpha, (const T*)add_c, alpha_c,
                         C.nrhs, (int)trans, partial, (const int32_t*)it.mlist, skip, (const T*)C.d_zero_tile);
    }
  } else {
    hipLaunchKernelGGL((k_tile_mv<T, NV, NB16, CLS, LD>), dim3((unsigned)grid), dim3(256), 0, s, it.n, it.d,
                       C.d_subs, tiles, (const T*)in, (T*)out, (const T*)add, alpha, (const T*)add_c, alpha_c,
                       C.nrhs, (int)trans, partial, (const int32_t*)it.mlist, skip, (const T*)C.d_zero_tile);
  }
  if (split)
    hipLaunchKernelGGL(k_mv_reduce<T>, dim3((unsigned)it.n_out), dim3(256), 0, s, it.n_out, it.outs, C.d_subs,
                       (const T*)partial, (T*)out, (const T*)add, alpha, (const T*)add_c, alpha_c, C.nrhs, skip);
}

template <class T, int CLS>
static void mv_dispatch(Ctx& C, hipStream_t s, const Items& it, bool trans, const void* in, void* out,
                        const void* add, T alpha, const void* add_c, T alpha_c, const int* skip) {
  const int nr = C.nrhs;
  // full RHS blocks (16, 32) take the instances with a compile-time stride
  if (nr == 1)
    mv_launch<T, 1, 0, CLS, 0>(C, s, it, trans, in, out, add, alpha, add_c, alpha_c, skip);
  else if (nr == 2)
    mv_launch<T, 2, 0, CLS, 0>(C, s, it, trans, in, out, add, alpha, add_c, alpha_c, skip);
  else if (nr <= 4)
    mv_launch<T, 4, 0, CLS, 0>(C, s, it, trans, in, out, add, alpha, add_c, alpha_c, skip);
  else if (nr <= 8)
    mv_launch<T, 8, 0, CLS, 0>(C, s, it, trans, in, out, add, alpha, add_c, alpha_c, skip);
  else if (nr == 16)
    mv_launch<T, 0, 1, CLS, 16>(C, s, it, trans, in, out, add, alpha, add_c, alpha_c, skip);
  else if (nr < 16)
    mv_launch<T, 0, 1, CLS, 0>(C, s, it, trans, in, out, add, alpha, add_c, alpha_c, skip);
  else if (nr == 32)
    mv_launch<T, 0, 2, CLS, 32>(C, s, it, trans, in, out, add, alpha, add_c, alpha_c, skip);
  else
    mv_launch<T, 0, 2, CLS, 0>(C, s, it, trans, in, out, add, alpha, add_c, alpha_c, skip);
}

// out = add + alpha * (product) on r-row output blocks, add_c + alpha_c *
// (product) on corner-row output blocks (forward passes only); side: launch
// on the side stream (not used while per-class timing is on)
template <class T>
static void mv(Ctx& C, const Items& it, bool trans, const void* in, void* out, const void* add, T alpha,
               const int* skip = nullptr, const void* add_c = nullptr, T alpha_c = (T)1, bool side = false) {
  if (it.n == 0) return;
  hipEvent_t e0, e1;
  bool timed = prof_begin(C, item_class(C, it), &e0, &e1);
  hipStream_t s = side ? C.st2 : C.st;
  const int cls = item_class(C, it);
  if (cls == DD_PROF_FULL)
    mv_dispatch<T, DD_PROF_FULL>(C, s, it, trans, in, out, add, alpha, add_c, alpha_c, skip);
  else if (cls == DD_PROF_CROSS)
    mv_dispatch<T, DD_PROF_CROSS>(C, s, it, trans, in, out, add, alpha, add_c, alpha_c, skip);
  else if (cls == DD_PROF_CORNER)
    mv_dispatch<T, DD_PROF_CORNER>(C, s, it, trans, in, out, add, alpha, add_c, alpha_c, skip);
  else
    mv_dispatch<T, DD_PROF_COARSE>(C, s, it, trans, in, out, add, alpha, add_c, alpha_c, skip);
  if (timed) HIPCHK(hipEventRecord(e1, C.st));
}

// fork: work queued on st so far is visible to the side stream; join: the
// side stream's work is visible to everything queued on st afterwards
// Right-hand sides per lane in the vector forms of the multiplier-space
// kernels (k_*_v): 4 when nrhs is a multiple of 4, else 2 when even, else
// the scalar forms.
static int vec_width(int nr) { return nr % 4 == 0 ? 4 : (nr % 2 == 0 ? 2 : 1); }

// per-RHS block partials of x . y over n rows [n][nrhs] (kDotBlocks blocks)
static void dot_partial(Ctx& C, hipStream_t st, int64_t n, const double* x, const double* y, double* partial,
                        const int* skip) {
  const int nr = C.nrhs, V = vec_width(nr);
  if (V == 4)
    hipLaunchKernelGGL((k_dot_partial_v<4>), dim3(kDotBlocks), dim3(256), 0, st, n, x, y, nr, partial, skip);
  else if (V == 2)
    hipLaunchKernelGGL((k_dot_partial_v<2>), dim3(kDotBlocks), dim3(256), 0, st, n, x, y, nr, partial, skip);
  else
    hipLaunchKernelGGL(k_dot_partial, dim3(kDotBlocks), dim3(256), 0, st, n, x, y, nr, partial, skip);
}

// v[rows[k]] = sign * p[lam[k]] (B_s^T p on the listed interface rows); with
// add: v = add - sign * p
template <class T>
static void lambda_gather(Ctx& C, int64_t n, const int32_t* lam, const double* p, T* v, const int* skip,
                          const T* add = nullptr) {
  const int nr = C.nrhs, V = vec_width(nr);
  hipStream_t st = C.st;
  if (V == 4)
    hipLaunchKernelGGL((k_lambda_gather_v<T, 4>), dim3(nblk(n * nr / 4)), dim3(256), 0, st, n, C.d_grow, lam, p, v,
                       nr, skip, add);
  else if (V == 2)
    hipLaunchKernelGGL((k_lambda_gather_v<T, 2>), dim3(nblk(n * nr / 2)), dim3(256), 0, st, n, C.d_grow, lam, p, v,
                       nr, skip, add);
  else
    hipLaunchKernelGGL(k_lambda_gather<T>, dim3(nblk(n * nr)), dim3(256), 0, st, n, C.d_grow, lam, p, v, nr, skip,
                       add);
}

// coarse rows of y = (add) + sum over each corner's subdomain rows of x
template <class T>
static void coarse_gather(Ctx& C, hipStream_t st, const T* x, T* y, const T* add, const int* skip) {
  const int nr = C.nrhs, V = vec_width(nr);
  const int64_t n = (int64_t)C.Kc * NB;
  if (V == 4)
    hipLaunchKernelGGL((k_coarse_gather_v<T, 4>), dim3(nblk(n * nr / 4)), dim3(256), 0, st, n, C.coarse_row0,
                       C.d_cgptr, C.d_cgrows, x, y, add, nr, skip);
  else if (V == 2)
    hipLaunchKernelGGL((k_coarse_gather_v<T, 2>), dim3(nblk(n * nr / 2)), dim3(256), 0, st, n, C.coarse_row0,
                       C.d_cgptr, C.d_cgrows, x, y, add, nr, skip);
  else
    hipLaunchKernelGGL(k_coarse_gather<T>, dim3(nblk(n * nr)), dim3(256), 0, st, n, C.coarse_row0, C.d_cgptr,
                       C.d_cgrows, x, y, add, nr, skip);
}

// subdomain corner rows of x = scale * their coarse rows of z
template <class T>
static void corner_scatter(Ctx& C, hipStream_t st, const T* z, T* x, T scale, const int* skip) {
  const int nr = C.nrhs, V = vec_width(nr);
  const int64_t n = C.n_csc;
  if (V == 4)
    hipLaunchKernelGGL((k_corner_scatter_v<T, 4>), dim3(nblk(n * nr / 4)), dim3(256), 0, st, n, C.d_cscrows,
                       C.d_csccrow, z, x, scale, nr, skip);
  else if (V == 2)
    hipLaunchKernelGGL((k_corner_scatter_v<T, 2>), dim3(nblk(n * nr / 2)), dim3(256), 0, st, n, C.d_cscrows,
                       C.d_csccrow, z, x, scale, nr, skip);
  else
    hipLaunchKernelGGL(k_corner_scatter<T>, dim3(nblk(n * nr)), dim3(256), 0, st, n, C.d_cscrows, C.d_csccrow, z,
                       x, scale, nr, skip);
}

// Fp = sum_s B_s (u + u2) with the partials of p . Fp (p may be null)
template <class T>
static void scatter_dot(Ctx& C, const T* u, const T* u2, double* Fp, const double* p, const int* skip) {
  const int nr = C.nrhs, V = vec_width(nr);
  hipStream_t st = C.st;
  if (V == 4)
    hipLaunchKernelGGL((k_scatter_dot_v<T, 4>), dim3(kDotBlocks), dim3(256), 0, st, C.nlam, C.d_lrow0, C.d_lrow1, u,
                       u2, Fp, p, nr, C.d_partial, skip);
  else if (V == 2)
    hipLaunchKernelGGL((k_scatter_dot_v<T, 2>), dim3(kDotBlocks), dim3(256), 0, st, C.nlam, C.d_lrow0, C.d_lrow1, u,
                       u2, Fp, p, nr, C.d_partial, skip);
  else
    hipLaunchKernelGGL(k_scatter_dot<T>, dim3(kDotBlocks), dim3(256), 0, st, C.nlam, C.d_lrow0, C.d_lrow1, u, u2,
                       Fp, p, nr, C.d_partial, skip);
}

static void fork_side(Ctx& C) {
  HIPCHK(hipEventRecord(C.ev_fork, C.st));
  HIPCHK(hipStreamWaitEvent(C.st2, C.ev_fork, 0));
}
static void join_side(Ctx& C) {
  HIPCHK(hipEventRecord(C.ev_join, C.st2));
  HIPCHK(hipStreamWaitEvent(C.st, C.ev_join, 0));
}

// The symmetric product M in into the partial slots, and the reduce of the
// slots: out (interface rows) = add + M in.  The per-class timing of
// DD_PROF_SCHUR covers this kernel alone: its events are attached to the
// kernel's dispatch (start and end of its execution).
template <class T>
static void symv_product(Ctx& C, const void* in, const int* skip, hipStream_t s) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool timed = prof_begin(C, DD_PROF_SCHUR, &e0, &e1, false);
  int64_t ng = (C.sym.n + 3) / 4;
  if (C.tuning.sym_persist > 0) ng = std::min<int64_t>(ng, C.tuning.sym_persist);
  const dim3 grid((unsigned)ng);
  // a full RHS block (16 or 32) takes the instance with a compile-time stride
  // (timing happens in eager steps only; captured steps launch plainly)
#define DD_SYMV_ARGS                                                                                      \
  C.sym.n, C.sym.d, C.d_subs, C.d_m_off, (const T*)C.d_mtri, (const T*)in, (T*)C.sym.partial, C.nrhs, skip, \
      (const T*)C.sym.zero
#define DD_SYMV_LD(NB16, PW, LD)                                                                       \
  do {                                                                                                 \
    if (timed)                                                                                         \
      hipExtLaunchKernelGGL((k_symv<T, NB16, PW, LD>), grid, dim3(256), 0, s, e0, e1, 0, DD_SYMV_ARGS); \
    else                                                                                               \
      hipLaunchKernelGGL((k_symv<T, NB16, PW, LD>), grid, dim3(256), 0, s, DD_SYMV_ARGS);              \
  } while (0)
#define DD_SYMV(NB16, PW)                \
  do {                                   \
    if (C.nrhs == 16 * (NB16))           \
      DD_SYMV_LD(NB16, PW, 16 * (NB16)); \
    else                                 \
      DD_SYMV_LD(NB16, PW, 0);           \
  } while (0)
  // panel width 4 exists for FP32 only (FP64 accumulators do not fit)
  bool pw4 = false;
  if constexpr (sizeof(T) == 4) {
    if (C.sym.pw == 4) {
      pw4 = true;
      if (C.nrhs <= 16)
        DD_SYMV(1, 4);
      else
        DD_SYMV(2, 4);
    }
  }
  if (!pw4) {
    if (C.nrhs <= 16)
      DD_SYMV(1, 2);
    else
      DD_SYMV(2, 2);
  }
#undef DD_SYMV
#undef DD_SYMV_LD
#undef DD_SYMV_ARGS
}

template <class T>
static void symv_reduce(Ctx& C, void* out, const void* add, const int* skip, hipStream_t s) {
  hipLaunchKernelGGL(k_mv_reduce<T>, dim3((unsigned)C.sym.n_out), dim3(256), 0, s, C.sym.n_out, C.sym.outs,
                     C.d_subs, (const T*)C.sym.partial, (T*)out, (const T*)add, (T)1, (const T*)nullptr, (T)1,
                     C.nrhs, skip);
}

// out (interface rows) = M in
template <class T>
static void symv(Ctx& C, const void* in, void* out, const int* skip, bool side) {
  if (C.sym.n == 0) return;
  hipStream_t s = side ? C.st2 : C.st;
  symv_product<T>(C, in, skip, s);
  symv_reduce<T>(C, out, nullptr, skip, s);
}

// coarse: y rows of Xin (coarse block) -> Xout coarse rows = K_cc^-1 y via
// Linv then Linv^T (tmp holds the intermediate)
template <class T>
static void coarse_solve(Ctx& C, void* Xin, void* Xtmp, void* Xout, const int* skip) {
  mv<T>(C, C.co_N, false, Xin, Xtmp, nullptr, (T)1, skip);
  mv<T>(C, C.co_T, true, Xtmp, Xout, nullptr, (T)1, skip);
}

// F p -> Fp (uses X5..X8):
//   v = B_s^T p;  y = Psi_G v (corner rows);  z = K_cc^-1 sum B_c^T y;
//   u = M v + Psi_G^T z with M = Linv_GG^T Linv_GG;  F p = sum B_s u
// M v needs only v: it runs on the side stream while the corner rows and
// the coarse chain run on st (disjoint rows of X5 / X6 / X8, own partial
// slots).
// gathered: X5 already holds v = B_s^T p (the CG iteration writes it while
// updating p)
// X8 = M X5 + Psi_G^T z, z = K_cc^-1 sum_s B_c^T Psi_G X5: the local
// interface response to the interface loads held in the interface rows of X5
template <class T>
static void apply_local(Ctx& C, const int* skip) {
  const int nr = C.nrhs;
  hipStream_t st = C.st;
  void **X = C.X;
  const bool overlap = C.Kc > 0 && !C.prof;
  if (overlap) fork_side(C);
  // the corner rows are submitted first, so that the chain on st (the longer
  // one) gets its workgroups dispatched ahead of the symmetric product's
  // (graded 48^3: 16.1 -> 15.5 ms/step; 64^3 unchanged)
  if (C.Kc > 0) mv<T>(C, C.corner_N, false, X[5], X[6], nullptr, (T)1, skip);
  symv<T>(C, X[5], X[8], skip, overlap);
  if (C.Kc > 0) {
    coarse_gather<T>(C, st, (const T*)X[6], (T*)X[6], nullptr, skip);
    coarse_solve<T>(C, X[6], X[7], X[5], skip);
    corner_scatter<T>(C, st, (const T*)X[5], (T*)X[6], (T)1, skip);
  }
  // Psi_G^T z goes to its own buffer (rows of subdomains without corners
  // stay zero from setup), so it does not wait for M v; consumers add X9
  if (C.Kc > 0) mv<T>(C, C.corner_T, true, X[6], X[9], nullptr, (T)1, skip);
  if (overlap) join_side(C);
}

// The interface and corner part of a local solve (pre-solve and recovery),
// from u on the interface rows of `u` and the corner loads g' on the corner
// rows of `gp`:
//   x_c = K_cc^-1 sum_s B_c^T (g' - Psi_G u)       (coarse rows of xc)
//   out = M u - Psi_G^T x_c                          (interface rows of out)
// With L_rr^-1 split by the column blocks of the factor, this is the
// interface and corner part of K_rr^-1 applied to the subdomain loads after
// the interior elimination: M u = L_GG^-T L_GG^-1 u, and Psi_G = L_cG L_GG^-1
// carries the corner coupling.  M u runs on the side stream beside the
// corner chain (X6, X7, X9), as in apply_local; out may be u (the product
// has read u before the reduce writes out).
template <class T>
static void interface_local(Ctx& C, void* u, const void* gp, void* out, void* xc, const int* skip) {
  void** X = C.X;
  const bool overlap = C.Kc > 0 && C.sym.n > 0 && !C.prof;
  if (overlap) fork_side(C);
  // corner rows first, as in apply_local
  if (C.Kc > 0) mv<T>(C, C.corner_N, false, u, X[6], nullptr, (T)1, skip, gp, (T)-1);
  if (C.sym.n > 0) symv_product<T>(C, u, skip, overlap ? C.st2 : C.st);
  if (C.Kc > 0) {
    // corner rows of X6: g' - Psi_G u (above); their coarse sum; x_c = K_cc^-1 (.)
    coarse_gather<T>(C, C.st, (const T*)X[6], (T*)X[6], nullptr, skip);
    coarse_solve<T>(C, X[6], X[7], xc, skip);
    // -x_c on the corner rows of X6; X9 = -Psi_G^T x_c
    corner_scatter<T>(C, C.st, (const T*)xc, (T*)X[6], (T)-1, skip);
    mv<T>(C, C.corner_T, true, X[6], X[9], nullptr, (T)1, skip);
  }
  if (overlap) join_side(C);
  if (C.sym.n > 0) symv_reduce<T>(C, out, C.Kc > 0 ? X[9] : nullptr, skip, C.st);
}

// the second part of the local response (X9) when there is one
static const void* corner_part(const Ctx& C) { return C.Kc > 0 ? C.X[9] : nullptr; }

template <class T>
static void apply_F(Ctx& C, const double* p, double* Fp, const int* skip, bool dot = false, bool gathered = false) {
  const int nr = C.nrhs;
  hipStream_t st = C.st;
  void **X = C.X;
  if (!gathered)
    lambda_gather<T>(C, C.n_grow, C.d_glam, p, (T*)X[5], skip);
  apply_local<T>(C, skip);
  scatter_dot<T>(C, (const T*)X[8], (const T*)corner_part(C), Fp, dot ? p : (const double*)nullptr, skip);
}

// y = (lam + lam(partner side)) - R (U + U2) over the n side rows (lam may
// be null), four or two right-hand sides per thread when nrhs allows
template <class T>
static void robin_apply(Ctx& C, int64_t n, const double* lam, const T* U, const T* U2, double* y, const int* skip) {
  const int nr = C.nrhs, V = vec_width(nr);
  hipStream_t st = C.st;
  if (V == 4)
    hipLaunchKernelGGL((k_robin_apply_v<T, 4>), dim3(nblk(n * nr / 4)), dim3(256), 0, st, n, C.d_rrp, C.d_rrow,
                       C.d_rval, C.d_partner2, lam, U, U2, y, nr, skip);
  else if (V == 2)
    hipLaunchKernelGGL((k_robin_apply_v<T, 2>), dim3(nblk(n * nr / 2)), dim3(256), 0, st, n, C.d_rrp, C.d_rrow,
                       C.d_rval, C.d_partner2, lam, U, U2, y, nr, skip);
  else
    hipLaunchKernelGGL(k_robin_apply<T>, dim3(nblk(n * nr)), dim3(256), 0, st, n, C.d_rrp, C.d_rrow, C.d_rval,
                       C.d_partner2, lam, U, U2, y, nr, skip);
}

// Robin variant: y = G lam = lam + lam(partner side) - R (x_G response of
// the other side), with the response of every side computed by apply_local;
// every kernel returns at once while *skip != 0
template <class T>
static void apply_G(Ctx& C, const double* lam, double* y, const int* skip) {
  const int nr = C.nrhs;
  const int64_t n = C.n_grow, nl = n * nr;
  hipStream_t st = C.st;
  lambda_gather<T>(C, n, C.d_code2, lam, (T*)C.X[5], skip);
  apply_local<T>(C, skip);
  robin_apply<T>(C, n, lam, (const T*)C.X[8], (const T*)corner_part(C), y, skip);
}

// the two projections of classical Gram-Schmidt (k_gm_project), for nv <= KMAX
template <bool FIRST>
static void gm_project(Ctx& C, int nv, double* w, const int* stop) {
  const int nr = C.nrhs;
  const int64_t n = C.n_grow, ldv = n * nr;
  hipStream_t st = C.st;
  const double* V = C.d_gmV;
  const double* ss = C.d_gm_st->ss;
  double* part = FIRST ? C.d_gm_partial : nullptr;
#define DD_GM_PROJECT(K)                                                                                      \
  hipLaunchKernelGGL((k_gm_project<K, FIRST>), dim3(kDotBlocks), dim3(256), 0, st, n, nv, V, ldv,             \
                     (const double*)C.d_gm_h, w, nr, part, ss, stop)
  if (nv <= 8 && nr % 2 == 0)
    // two right-hand sides per lane (a wider form holds too many registers)
    hipLaunchKernelGGL((k_gm_project_v<8, FIRST, 2>), dim3(kDotBlocks), dim3(256), 0, st, n, nv, V, ldv,
                       (const double*)C.d_gm_h, w, nr, part, ss, stop);
  else if (nv <= 8)
    DD_GM_PROJECT(8);
  else if (nv <= 16)
    DD_GM_PROJECT(16);
  else if (nv <= 24)
    DD_GM_PROJECT(24);
  else if (nv <= 32)
    DD_GM_PROJECT(32);
  else
    DD_GM_PROJECT(kGmresRestart);
#undef DD_GM_PROJECT
}

// iteration j of the device GMRES (basis V_0 .. V_j, new vector w = V_{j+1}):
// w = G V_j; classical Gram-Schmidt applied twice, in three passes over the
// basis (the dots of the first projection; its update fused with the dots of
// the second; the second update fused with the normalisation, whose norm
// |w''|^2 = |w'|^2 - |h2|^2 comes from the second dots); the Givens update
// of every open RHS in between.  Every kernel returns at once once the solve
// has stopped.
template <class T>
static void gmres_iteration(Ctx& C, int j) {
  const int nr = C.nrhs, m = kGmresRestart;
  hipStream_t st = C.st;
  const int64_t n = C.n_grow, nl = n * nr, ldv = nl;
  double* V = C.d_gmV;
  double* w = V + (int64_t)(j + 1) * ldv;
  GmState* gs = C.d_gm_st;
  const int* stop = &gs->stop;
  apply_G<T>(C, V + (int64_t)j * ldv, w, stop);
  // h1 = [V_0 .. V_j, w]^T w (the last entry, |w|^2, is not used)
  if (vec_width(nr) == 4)
    hipLaunchKernelGGL((k_mdot_v<4>), dim3(kDotBlocks, (j + 2 + kMdotChunk - 1) / kMdotChunk), dim3(256), 0, st, n,
                       j + 2, (const double*)V, ldv, (const double*)w, nr, C.d_gm_partial, stop);
  else if (vec_width(nr) == 2)
    hipLaunchKernelGGL((k_mdot_v<2>), dim3(kDotBlocks, (j + 2 + kMdotChunk - 1) / kMdotChunk), dim3(256), 0, st, n,
                       j + 2, (const double*)V, ldv, (const double*)w, nr, C.d_gm_partial, stop);
  else
    hipLaunchKernelGGL(k_mdot, dim3(kDotBlocks, (j + 2 + kMdotChunk - 1) / kMdotChunk), dim3(256), 0, st, n, j + 2,
                       (const double*)V, ldv, (const double*)w, nr, C.d_gm_partial, stop);
  hipLaunchKernelGGL(k_mdot_reduce, dim3(j + 2), dim3(256), 0, st, j + 2, nr, kDotBlocks,
                     (const double*)C.d_gm_partial, C.d_gm_h, C.d_gm_tot, 1, stop);
  // w' = w - V h1 with h2 = V^T w' and |w'|^2
  gm_project<true>(C, j + 1, w, stop);
  hipLaunchKernelGGL(k_mdot_reduce, dim3(j + 2), dim3(256), 0, st, j + 2, nr, kDotBlocks,
                     (const double*)C.d_gm_partial, C.d_gm_h, C.d_gm_tot, 0, stop);
  hipLaunchKernelGGL(k_gm_givens, dim3(1), dim3(kScalarThreads), 0, st, j, nr, (const double*)C.d_gm_h,
                     (const double*)C.d_gm_tot, gs, C.d_gm_H, C.d_gm_cs, C.d_gm_sn, C.d_gm_g, m, C.opt.cg_tol,
                     C.opt.cg_max_iter, stop);
  // w'' = (w' - V h2) / |w''|
  gm_project<false>(C, j + 1, w, stop);
}

// Restarted GMRES on G lam = rhs (Sec. III-B's multiplier system for the
// edge-only unknowns), all right-hand sides in lock step, with its scalar
// work on the device (k_gm_*): the host launches blocks of check_every
// iterations (replayed from captured graphs when the stream allows) and reads
// the small state back once per block.  Stop when ||rhs - G lam|| <= tol
// ||rhs|| for every RHS (or at the iteration cap).  The rhs is -R x0 with x0
// the interface rows of the pre-solve (X4).
template <class T>
static int dp2_gmres(Ctx& C, int* iters, double* relres) {
  const int nr = C.nrhs;
  hipStream_t st = C.st;
  const int64_t n = C.n_grow, nl = n * nr, ldv = nl;
  const int m = kGmresRestart;
  double* V = C.d_gmV;
  GmState* gs = C.d_gm_st;
  const int cap = C.opt.cg_max_iter;
  const int chk = std::max(1, std::min(C.opt.check_every, m));
  const int nblocks = (m + chk - 1) / chk;
  robin_apply<T>(C, n, nullptr, (const T*)C.X[4], (const T*)nullptr, C.d_gm_rhs, nullptr);
  hipLaunchKernelGGL(k_zero<double>, dim3(nblk(nl)), dim3(256), 0, st, nl, C.d_lam2, (const int*)nullptr);
  dot_partial(C, st, n, (const double*)C.d_gm_rhs, (const double*)C.d_gm_rhs, C.d_gm_wpart, nullptr);
  hipLaunchKernelGGL(k_gm_init, dim3(1), dim3(kScalarThreads), 0, st, nr, (const double*)C.d_gm_wpart, gs);
  auto read_state = [&]() {
    HIPCHK(hipMemcpyAsync(C.h_gm_st, gs, sizeof(GmState), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  };
  read_state();
  const bool graph = C.opt.use_graph && st != nullptr && !C.prof;
  if (graph && (int)C.gm_graphs.size() != nblocks) {
    for (hipGraphExec_t g : C.gm_graphs)
      if (g) HIPCHK(hipGraphExecDestroy(g));
    C.gm_graphs.assign(nblocks, nullptr);
  }
  while (!C.h_gm_st->stop) {
    // r0 = rhs - G lam in V_0 (lam = 0 on the first cycle), |r0| e_1, V_0 = r0 / |r0|
    if (C.h_gm_st->total == 0) {
      hipLaunchKernelGGL(k_copy, dim3(nblk(nl)), dim3(256), 0, st, nl, (const double*)C.d_gm_rhs, V,
                         (const int*)nullptr);
    } else {
      apply_G<T>(C, C.d_lam2, V, nullptr);
      hipLaunchKernelGGL(k_rsub, dim3(nblk(nl)), dim3(256), 0, st, nl, (const double*)C.d_gm_rhs, V);
    }
    dot_partial(C, st, n, (const double*)V, (const double*)V, C.d_gm_wpart, nullptr);
    hipLaunchKernelGGL(k_gm_cycle, dim3(1), dim3(kScalarThreads), 0, st, nr, (const double*)C.d_gm_wpart, gs,
                       C.d_gm_g, m, cap);
    hipLaunchKernelGGL(k_vnormalize, dim3(nblk(nl)), dim3(256), 0, st, n, (const double*)V, (const double*)gs->ss,
                       V, nr, (const int*)nullptr);
    for (int b = 0; b < nblocks; ++b) {
      const int j0 = b * chk, j1 = std::min(m, j0 + chk);
      if (graph) {
        if (!C.gm_graphs[b]) {
          HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
          hipGraph_t g = nullptr;
          try {
            for (int j = j0; j < j1; ++j) gmres_iteration<T>(C, j);
          } catch (...) {
            (void)hipStreamEndCapture(st, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
          }
          HIPCHK(hipStreamEndCapture(st, &g));
          hipError_t e = hipGraphInstantiate(&C.gm_graphs[b], g, nullptr, nullptr, 0);
          (void)hipGraphDestroy(g);
          HIPCHK(e);
        }
        HIPCHK(hipGraphLaunch(C.gm_graphs[b], st));
      } else {
        for (int j = j0; j < j1; ++j) gmres_iteration<T>(C, j);
      }
      HIPCHK(hipGetLastError());
      read_state();
      if (C.h_gm_st->stop) break;
    }
    // lam += V y, y from the triangular systems of each RHS's first cols columns
    hipLaunchKernelGGL(k_gm_solve, dim3(1), dim3(kScalarThreads), 0, st, nr, gs, (const double*)C.d_gm_H,
                       (const double*)C.d_gm_g, C.d_gm_y, m);
    hipLaunchKernelGGL(k_mupdate, dim3(nblk(nl)), dim3(256), 0, st, n, m, (const double*)V, ldv,
                       (const double*)C.d_gm_y, 1.0, C.d_lam2, nr, (const int*)&gs->jmax);
    // a cycle that ran out of columns restarts unless the cap is reached
    if (!C.h_gm_st->stop && C.h_gm_st->total >= cap) break;
  }
  HIPCHK(hipGetLastError());
  const GmState& hs = *C.h_gm_st;
  bool all = true;
  for (int r = 0; r < nr; ++r) {
    iters[r] = hs.iters[r];
    relres[r] = hs.relres[r];
    if (!hs.conv[r]) all = false;
  }
  return all ? DD_OK : DD_ERR_NO_CONVERGENCE;
}

static void dot_to_host(Ctx& C, const double* x, const double* y, int64_t n, double* out) {
  dot_partial(C, C.st, n, x, y, C.d_partial, nullptr);
  HIPCHK(hipMemcpyAsync(C.h_partial, C.d_partial, sizeof(double) * kDotBlocks * kMaxRhs, hipMemcpyDeviceToHost,
                        C.st));
  HIPCHK(hipStreamSynchronize(C.st));
  for (int r = 0; r < C.nrhs; ++r) {
    double s = 0.0;
    for (int b = 0; b < kDotBlocks; ++b) s += C.h_partial[b * kMaxRhs + r];
    out[r] = s;
  }
}

// z = K_lam r (the lumped preconditioner) with the r.z and r.r partials.
// Vector form for even nrhs: at 16 RHS, four per lane, one row in flight,
// nonzeros in batches of 4 (16.60 -> 16.17 ms/step at 64^3 with 16 RHS;
// one row in batches of 8 the same, two rows spill).  Scalar form: two rows
// in flight per lane, their nonzeros in batches of 8 (batches of 12 spilled:
// 19.65 against 19.40 ms/step; one row of 12: 19.75; four rows of 6: 20.02)
static void lam_precond(Ctx& C, const int* skip) {
  const int nr = C.nrhs;
  if (vec_width(nr) == 4)
    hipLaunchKernelGGL((k_lam_precond_v<1, 4, 4>), dim3(kDotBlocks), dim3(256), 0, C.st, C.nlam, C.d_lrp, C.d_lci,
                       C.d_lvals, (const double*)C.d_res, C.d_z, nr, C.d_partial, C.d_partial2, skip);
  else if (vec_width(nr) == 2)
    hipLaunchKernelGGL((k_lam_precond_v<2, 4, 2>), dim3(kDotBlocks), dim3(256), 0, C.st, C.nlam, C.d_lrp, C.d_lci,
                       C.d_lvals, (const double*)C.d_res, C.d_z, nr, C.d_partial, C.d_partial2, skip);
  else
    hipLaunchKernelGGL((k_lam_precond<2, 8>), dim3(kDotBlocks), dim3(256), 0, C.st, C.nlam, C.d_lrp, C.d_lci,
                       C.d_lvals, (const double*)C.d_res, C.d_z, nr, C.d_partial, C.d_partial2, skip);
}

// x = A^-1 b (one decomposed solve, unknown-major [nint][nrhs] FP64).
// Returns DD_OK or DD_ERR_NO_CONVERGENCE; fills iters/relres.
// Captured form (fixed_iters > 0, inside a stream capture): exactly
// fixed_iters CG iterations (kernels return at once after convergence), no
// host synchronisation and no warm start; every kernel is skipped while
// *gate != 0; the CG state is snapshotted into C.d_rs slot `slot` and
// iters/relres are not filled (read back with the step).
template <class T>
static int dd_solve_once(Ctx& C, const double* b, double* x, Ctx::Warm* warm, int* iters, double* relres,
                         const int* gate = nullptr, int fixed_iters = 0, int slot = 0) {
  const int nr = C.nrhs;
  hipStream_t st = C.st;
  void** X = C.X;
  const T one = 1, mone = -1;
  // ---- pre-solve --------------------------------------------------------
  const bool captured = fixed_iters > 0;
  if (captured && (warm || C.opt.method == 1))
    throw DDError{DD_ERR_STATE, "captured solve: no warm start, first variant only"};
  if (vec_width(nr) == 4)
    hipLaunchKernelGGL((k_split_v<T, 4>), dim3(nblk(C.rows_total * nr / 4)), dim3(256), 0, st, C.rows_total,
                       C.d_rowsrc, b, (T*)X[0], nr, gate);
  else if (vec_width(nr) == 2)
    hipLaunchKernelGGL((k_split_v<T, 2>), dim3(nblk(C.rows_total * nr / 2)), dim3(256), 0, st, C.rows_total,
                       C.d_rowsrc, b, (T*)X[0], nr, gate);
  else
    hipLaunchKernelGGL(k_split<T>, dim3(nblk(C.rows_total * nr)), dim3(256), 0, st, C.rows_total, C.d_rowsrc, b,
                       (T*)X[0], nr, gate);
  // Through the column blocks of the factor store (L_rr^-1 = [L_II^-1, 0;
  // -L_GG^-1 L_GI L_II^-1, L_GG^-1]):
  //   t_I = L_II^-1 w_I                                  (X1, I rows)
  //   y_G = w_G - L_GI t_I,  g' = w_c - L_cI t_I        (X2, Gamma and corner rows)
  // both kept for the recovery; then the interface part with M = L_GG^-T
  // L_GG^-1 and Psi_G = L_cG L_GG^-1:
  //   z0 = K_cc^-1 sum B_c^T (g' - Psi_G y_G),  X4 = M y_G - Psi_G^T z0
  // (the d-contribution of every subdomain)
  mv<T>(C, C.full_N, false, X[0], X[1], nullptr, one, gate);
  mv<T>(C, C.cross_N, false, X[1], X[2], X[0], mone, gate, X[0], mone);
  interface_local<T>(C, X[2], X[2], X[4], X[3], gate);
  for (int r = 0; r < nr; ++r) {
    iters[r] = 0;
    relres[r] = 0.0;
  }
  int status = DD_OK;
  if (C.nlam > 0 && C.opt.method == 1) {
    // ---- Robin variant: GMRES on the per-side multipliers, then the same
    // recovery with each subdomain's own multipliers as interface loads
    status = dp2_gmres<T>(C, iters, relres);
    lambda_gather<T>(C, C.n_grow, C.d_code2, (const double*)C.d_lam2, (T*)X[5], nullptr, (const T*)X[2]);
  } else if (C.nlam > 0) {
    const int64_t nl = C.nlam * nr;
    scatter_dot<T>(C, (const T*)X[4], (const T*)nullptr, C.d_d, (const double*)nullptr, gate);
    // ---- CG on F lambda = d (stage 0 of k_cg_scalar resets the whole state) ----
    dot_partial(C, st, C.nlam, C.d_d, C.d_d, C.d_partial, gate);
    hipLaunchKernelGGL(k_cg_scalar, dim3(1), dim3(kScalarThreads), 0, st, 0, nr, (const double*)C.d_partial,
                       (const double*)nullptr, C.d_cg, C.opt.cg_tol, gate);
    hipLaunchKernelGGL(k_copy, dim3(nblk(nl)), dim3(256), 0, st, nl, (const double*)C.d_d, C.d_res, gate);
    if (warm && warm->have > 0) {
      if (C.opt.warm_start == 2 && warm->have >= 2)
        hipLaunchKernelGGL(k_extrap, dim3(nblk(nl)), dim3(256), 0, st, nl, (const double*)warm->cur,
                           (const double*)warm->old, C.d_lam);
      else
        HIPCHK(hipMemcpyAsync(C.d_lam, warm->cur, nl * sizeof(double), hipMemcpyDeviceToDevice, st));
      apply_F<T>(C, C.d_lam, C.d_Fp, nullptr);
      hipLaunchKernelGGL(k_sub, dim3(nblk(nl)), dim3(256), 0, st, nl, C.d_d, C.d_Fp, C.d_res);
      dot_partial(C, st, C.nlam, C.d_res, C.d_res, C.d_partial, nullptr);
      hipLaunchKernelGGL(k_cg_scalar, dim3(1), dim3(kScalarThreads), 0, st, 3, nr, (const double*)C.d_partial,
                         (const double*)nullptr, C.d_cg, C.opt.cg_tol, (const int*)nullptr);
    } else {
      hipLaunchKernelGGL(k_zero<double>, dim3(nblk(nl)), dim3(256), 0, st, nl, C.d_lam, gate);
    }
    // p = z = K_lam r (lumped preconditioner), or p = r
    const bool pre = C.opt.precond == 1 && C.lam_nnz > 0;
    if (pre) {
      lam_precond(C, gate);
      hipLaunchKernelGGL(k_cg_scalar, dim3(1), dim3(kScalarThreads), 0, st, 4, nr, (const double*)C.d_partial,
                         (const double*)nullptr, C.d_cg, C.opt.cg_tol, gate);
    }
    hipLaunchKernelGGL(k_copy, dim3(nblk(nl)), dim3(256), 0, st, nl, (const double*)(pre ? C.d_z : C.d_res), C.d_p,
                       gate);
    // v = B_s^T p for the first F application, padding rows zeroed (later
    // ones are written by k_cg_p_scatter, which leaves padding rows alone)
    lambda_gather<T>(C, C.n_grow, C.d_glam, (const double*)C.d_p, (T*)X[5], gate);
    const int* done = &C.d_cg->done;
    int it = 0;
    // an even block of iterations, so that every replay starts on p = d_p
    const int chk = std::max(2, (C.opt.check_every + 1) / 2 * 2);
    // no host check before the first block: its kernels return at once when
    // every RHS has converged already
    bool converged = false, have_state = false;
    // CG iteration k (p alternating between d_p and d_p2); every kernel
    // returns at once when all RHS have converged
    auto iteration = [&](int k) {
      double* pc = (k & 1) ? C.d_p2 : C.d_p;
      double* pn = (k & 1) ? C.d_p : C.d_p2;
      apply_F<T>(C, pc, C.d_Fp, done, true, true);
      hipLaunchKernelGGL(k_cg_scalar, dim3(1), dim3(kScalarThreads), 0, st, 1, nr, (const double*)C.d_partial,
                         (const double*)nullptr, C.d_cg, C.opt.cg_tol, (const int*)nullptr);
      if (pre) {
        if (vec_width(nr) == 4)
          hipLaunchKernelGGL((k_cg_xr_v<4>), dim3(nblk(nl / 4)), dim3(256), 0, st, C.nlam, nr, (const CgState*)C.d_cg,
                             (const double*)pc, (const double*)C.d_Fp, C.d_lam, C.d_res);
        else if (vec_width(nr) == 2)
          hipLaunchKernelGGL((k_cg_xr_v<2>), dim3(nblk(nl / 2)), dim3(256), 0, st, C.nlam, nr, (const CgState*)C.d_cg,
                             (const double*)pc, (const double*)C.d_Fp, C.d_lam, C.d_res);
        else
          hipLaunchKernelGGL(k_cg_xr, dim3(nblk(nl)), dim3(256), 0, st, C.nlam, nr, (const CgState*)C.d_cg,
                             (const double*)pc, (const double*)C.d_Fp, C.d_lam, C.d_res);
        lam_precond(C, done);
        hipLaunchKernelGGL(k_cg_scalar, dim3(1), dim3(kScalarThreads), 0, st, 2, nr, (const double*)C.d_partial,
                           (const double*)C.d_partial2, C.d_cg, C.opt.cg_tol, (const int*)nullptr);
      } else {
        hipLaunchKernelGGL(k_cg_xr_dot, dim3(kDotBlocks), dim3(256), 0, st, C.nlam, nr, (const CgState*)C.d_cg,
                           (const double*)pc, (const double*)C.d_Fp, C.d_lam, C.d_res, C.d_partial);
        hipLaunchKernelGGL(k_cg_scalar, dim3(1), dim3(kScalarThreads), 0, st, 2, nr, (const double*)C.d_partial,
                           (const double*)C.d_partial, C.d_cg, C.opt.cg_tol, (const int*)nullptr);
      }
      // p' and v = B_s^T p' in multiplier order (a gather over the interface
      // rows computed each p' twice: 19.65 against 19.40 ms/step)
      const double* base = pre ? C.d_z : C.d_res;
      if (vec_width(nr) == 4)
        hipLaunchKernelGGL((k_cg_p_scatter_v<T, 4>), dim3(nblk(nl / 4)), dim3(256), 0, st, C.nlam, C.d_lrow0,
                           C.d_lrow1, nr, (const CgState*)C.d_cg, base, (const double*)pc, pn, (T*)X[5]);
      else if (vec_width(nr) == 2)
        hipLaunchKernelGGL((k_cg_p_scatter_v<T, 2>), dim3(nblk(nl / 2)), dim3(256), 0, st, C.nlam, C.d_lrow0,
                           C.d_lrow1, nr, (const CgState*)C.d_cg, base, (const double*)pc, pn, (T*)X[5]);
      else
        hipLaunchKernelGGL(k_cg_p_scatter<T>, dim3(nblk(nl)), dim3(256), 0, st, C.nlam, C.d_lrow0, C.d_lrow1, nr,
                           (const CgState*)C.d_cg, base, (const double*)pc, pn, (T*)X[5]);
    };
    // captured step: a fixed number of iterations, the state snapshotted
    if (captured) {
      for (int k = 0; k < fixed_iters; ++k) iteration(k);
      hipLaunchKernelGGL(k_cg_snapshot, dim3(1), dim3(64), 0, st, slot, nr, (const CgState*)C.d_cg, C.d_rs, gate);
      converged = true;
      have_state = true;
    }
    // the block of chk iterations is captured once (fixed buffers, fixed
    // arguments) and replayed; needs a capturable (non-default) stream and
    // no per-launch event timing
    const bool graph = !captured && C.opt.use_graph && st != nullptr && !C.prof;
    if (graph && (!C.cg_graph || C.cg_graph_iters != chk)) {
      if (C.cg_graph) HIPCHK(hipGraphExecDestroy(C.cg_graph));
      C.cg_graph = nullptr;
      HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      for (int k = 0; k < chk; ++k) iteration(k);
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamEndCapture(st, &g));
      HIPCHK(hipGraphInstantiate(&C.cg_graph, g, nullptr, nullptr, 0));
      HIPCHK(hipGraphDestroy(g));
      C.cg_graph_iters = chk;
    }
    while (!captured && !converged && it < C.opt.cg_max_iter) {
      int todo = std::min(chk, C.opt.cg_max_iter - it);
      if (graph && todo == chk && (it & 1) == 0) {
        HIPCHK(hipGraphLaunch(C.cg_graph, st));
      } else {
        for (int k = 0; k < todo; ++k) iteration(it + k);
      }
      it += todo;
      HIPCHK(hipGetLastError());
      // the whole state, so that the last check also serves the report
      HIPCHK(hipMemcpyAsync(C.h_cg, C.d_cg, sizeof(CgState), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      have_state = true;
      converged = C.h_cg->done != 0;
    }
    if (!have_state) {
      HIPCHK(hipMemcpyAsync(C.h_cg, C.d_cg, sizeof(CgState), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
    }
    if (!captured) {
      const CgState& hs = *C.h_cg;
      for (int r = 0; r < nr; ++r) {
        iters[r] = hs.iters[r];
        relres[r] = hs.rr0[r] > 0 ? std::sqrt(hs.rr[r] / hs.rr0[r]) : 0.0;
      }
      if (!converged || hs.breakdown) status = DD_ERR_NO_CONVERGENCE;
    }
    if (warm) {
      std::swap(warm->cur, warm->old);
      HIPCHK(hipMemcpyAsync(warm->cur, C.d_lam, nl * sizeof(double), hipMemcpyDeviceToDevice, st));
      warm->have = std::min(2, warm->have + 1);
    }
    // ---- recovery -------------------------------------------------------------------
    // u = y_G - B_s^T lambda on the interface rows of X5
    lambda_gather<T>(C, C.n_grow, C.d_glam, (const double*)C.d_lam, (T*)X[5], gate, (const T*)X[2]);
  } else if (captured) {
    hipLaunchKernelGGL(k_cg_snapshot, dim3(1), dim3(64), 0, st, slot, nr, (const CgState*)C.d_cg, C.d_rs, gate);
  }
  // x_c = K_cc^-1 sum B_c^T (g' - Psi_G u) (coarse rows of X5, where the
  // collect reads corner unknowns), x_G = M u - Psi_G^T x_c (interface rows
  // of X5); u = y_G without multipliers
  interface_local<T>(C, C.nlam > 0 ? X[5] : X[2], X[2], X[5], X[5], gate);
  // x_c on the corner rows of X5; x_I = L_II^-T (t_I - L_GI^T x_G - L_cI^T x_c)
  if (C.Kc > 0) corner_scatter<T>(C, st, (const T*)X[5], (T*)X[5], one, gate);
  mv<T>(C, C.cross_T, true, X[5], X[2], X[1], mone, gate);
  mv<T>(C, C.full_T, true, X[2], X[5], nullptr, one, gate);
  if (vec_width(nr) == 4)
    hipLaunchKernelGGL((k_collect_v<T, 4>), dim3(nblk(C.P.nint * nr / 4)), dim3(256), 0, st, (int64_t)C.P.nint,
                       C.d_dsrc, (const T*)X[5], x, nr, gate);
  else if (vec_width(nr) == 2)
    hipLaunchKernelGGL((k_collect_v<T, 2>), dim3(nblk(C.P.nint * nr / 2)), dim3(256), 0, st, (int64_t)C.P.nint,
                       C.d_dsrc, (const T*)X[5], x, nr, gate);
  else
    hipLaunchKernelGGL(k_collect<T>, dim3(nblk(C.P.nint * nr)), dim3(256), 0, st, (int64_t)C.P.nint, C.d_dsrc,
                       (const T*)X[5], x, nr, gate);
  HIPCHK(hipGetLastError());
  return status;
}

// The global (T, S) product of k_csr (modes there): one thread per (row,
// RHS) for up to 4 RHS, the cooperative row groups for 5..32.
template <int G, int NB, int MODE>
static void csr_coop_launch(Ctx& C, hipStream_t st, const double* x1, const double* x2, const double* j1,
                            const double* j2, const double* z, double ca, double cb, double* y, double* y2,
                            const int* skip, double* y3) {
  const int64_t ni = C.P.nint;
  hipLaunchKernelGGL((k_csr_coop<G, NB, MODE>), dim3(nblk8(ni * G)), dim3(256), 0, st, ni, C.d_rp, C.d_ci, C.d_vals,
                     x1, x2, j1, j2, z, C.dt, ca, cb, y, y2, C.nrhs, skip, y3);
}

template <int G, int NB>
static void csr_coop_mode(Ctx& C, hipStream_t st, int mode, const double* x1, const double* x2, const double* j1,
                          const double* j2, const double* z, double ca, double cb, double* y, double* y2,
                          const int* skip, double* y3) {
  if (mode == 0)
    csr_coop_launch<G, NB, 0>(C, st, x1, x2, j1, j2, z, ca, cb, y, y2, skip, y3);
  else if (mode == 1)
    csr_coop_launch<G, NB, 1>(C, st, x1, x2, j1, j2, z, ca, cb, y, y2, skip, y3);
  else if (mode == 2)
    csr_coop_launch<G, NB, 2>(C, st, x1, x2, j1, j2, z, ca, cb, y, y2, skip, y3);
  else
    csr_coop_launch<G, NB, 3>(C, st, x1, x2, j1, j2, z, ca, cb, y, y2, skip, y3);
}

template <int G, int V, int NB>
static void csr_vec_mode(Ctx& C, hipStream_t st, int mode, const double* x1, const double* x2, const double* j1,
                         const double* j2, const double* z, double ca, double cb, double* y, double* y2,
                         const int* skip, double* y3) {
  const int64_t ni = C.P.nint;
#define DD_CSRV(M)                                                                                              \
  hipLaunchKernelGGL((k_csr_vec<G, V, NB, M>), dim3(nblk8(ni * G)), dim3(256), 0, st, ni, C.d_rp, C.d_ci, C.d_vals, \
                     x1, x2, j1, j2, z, C.dt, ca, cb, y, y2, C.nrhs, skip, y3)
  if (mode == 0)
    DD_CSRV(0);
  else if (mode == 1)
    DD_CSRV(1);
  else if (mode == 2)
    DD_CSRV(2);
  else
    DD_CSRV(3);
#undef DD_CSRV
}

static void csr_launch(Ctx& C, hipStream_t st, int mode, const double* x1, const double* x2, const double* j1,
                       const double* j2, const double* z, double ca, double cb, double* y, double* y2,
                       const int* skip = nullptr, double* y3 = nullptr) {
  const int nr = C.nrhs;
  const int64_t ni = C.P.nint;
  // 8, 16 and 32 RHS: the vector form, two right-hand sides per lane and
  // batches of 16 nonzeros (15.78 -> 15.45 ms/step at 64^3 with 16 RHS; four
  // per lane in batches of 8: 15.57, of 4: 15.60; two in batches of 8: 15.47)
  if (nr == 8)
    csr_vec_mode<4, 2, 16>(C, st, mode, x1, x2, j1, j2, z, ca, cb, y, y2, skip, y3);
  else if (nr == 16)
    csr_vec_mode<8, 2, 16>(C, st, mode, x1, x2, j1, j2, z, ca, cb, y, y2, skip, y3);
  else if (nr == 32)
    csr_vec_mode<16, 2, 16>(C, st, mode, x1, x2, j1, j2, z, ca, cb, y, y2, skip, y3);
  else if (nr <= 4)
    hipLaunchKernelGGL(k_csr, dim3(nblk8(ni * nr)), dim3(256), 0, st, mode, ni, C.d_rp, C.d_ci, C.d_vals, x1, x2, j1,
                       j2, z, C.dt, ca, cb, y, y2, nr, skip, y3);
  else if (nr <= 8)
    csr_coop_mode<8, 20>(C, st, mode, x1, x2, j1, j2, z, ca, cb, y, y2, skip, y3);
  else if (nr <= 16)
    csr_coop_mode<16, 20>(C, st, mode, x1, x2, j1, j2, z, ca, cb, y, y2, skip, y3);
  else
    csr_coop_mode<32, 20>(C, st, mode, x1, x2, j1, j2, z, ca, cb, y, y2, skip, y3);
}


// The refined solve of a step as one captured graph (x = A^-1 b, b and x
// internal buffers): |b|^2; solve 0; then for each captured sweep k the
// residual b - A x (FP64), its norm and the check against refine_tol on the
// device, the correction solve and x += delta, all skipped once the check
// passes; a last residual and check.  Each solve runs `iters` CG iterations
// (the kernels return at once after convergence).  One read-back after the
// graph gives the norms, the checks and every solve's CG state.  The
// graph goes into slot sg (which keeps its buffers and counts).  tx, sx
// (may be null): T x and S x of the accepted iterate, from its residual.
template <class T>
static void capture_step(Ctx& C, Ctx::StepGraph& sg, const double* b, double* x, double* tx, double* sx, int iters,
                         int sweeps) {
  hipStream_t st = C.st;
  const int nr = C.nrhs;
  const int64_t n = C.P.nint * nr;
  const double ca = C.beta * C.dt * C.dt, cb = (2 * C.beta - 1) * C.dt * C.dt;
  int it_dummy[kMaxRhs];
  double rr_dummy[kMaxRhs];
  HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  try {
    int* gate = reinterpret_cast<int*>(reinterpret_cast<char*>(C.d_rs) + offsetof(RefineState, gate));
    dot_partial(C, st, C.P.nint, b, b, C.d_rpart, nullptr);
    hipLaunchKernelGGL(k_refine_init, dim3(1), dim3(kScalarThreads), 0, st, nr, (const double*)C.d_rpart, C.d_rs);
    dd_solve_once<T>(C, b, x, nullptr, it_dummy, rr_dummy, gate, iters, 0);
    for (int k = 1; k <= sweeps + 1; ++k) {
      // only the last residual writes T x and S x (460 MB less at 64^3 with
      // 16 RHS), and it runs even when an earlier check has passed (x is
      // then the accepted iterate, the later sweeps being skipped), so T x
      // and S x always belong to the returned x.  Its norm and check stay
      // gated.  The residual arithmetic is the same in every pass (captured
      // and eager steps agree bit for bit).
      const bool last = k == sweeps + 1;
      csr_launch(C, st, 1, x, nullptr, nullptr, nullptr, b, ca, cb, C.g_r, last ? tx : nullptr,
                 last && tx ? nullptr : gate + (k - 1), last ? sx : nullptr);
      dot_partial(C, st, C.P.nint, (const double*)C.g_r, (const double*)C.g_r, C.d_rpart, gate + (k - 1));
      hipLaunchKernelGGL(k_refine_check, dim3(1), dim3(kScalarThreads), 0, st, k, nr, (const double*)C.d_rpart,
                         C.opt.refine_tol, C.d_rs, C.d_cg);
      if (k > sweeps) break;
      dd_solve_once<T>(C, C.g_r, C.g_t4, nullptr, it_dummy, rr_dummy, gate + k, iters, k);
      hipLaunchKernelGGL(k_axpy, dim3(nblk(n)), dim3(256), 0, st, n, 1.0, (const double*)C.g_t4, x,
                         (const int*)(gate + k));
    }
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(st, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamEndCapture(st, &g));
  if (sg.g) HIPCHK(hipGraphExecDestroy(sg.g));
  sg = Ctx::StepGraph{};
  hipError_t e = hipGraphInstantiate(&sg.g, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHK(e);
  sg.b = b;
  sg.x = x;
  sg.tx = tx;
  sg.sx = sx;
  sg.iters = iters;
  sg.sweeps = sweeps;
}

// A^-1 b with iterative refinement in the mixed form.  b, x: [nint][nrhs].
// what names the input of b in the message of a non-finite load.  With
// tx != nullptr the mixed form also leaves T x of the returned iterate there
// (from its last residual) and *tx_done is set; otherwise *tx_done = false.
template <class T>
static int solve_refined(Ctx& C, const double* b, double* x, Ctx::Warm* warm, dd_stats* stats,
                         const char* what = "b", double* tx = nullptr, bool* tx_done = nullptr,
                         bool step = false, double* sx = nullptr) {
  const int nr = C.nrhs;
  const int64_t n = C.P.nint * nr;
  hipStream_t st = C.st;
  const double ca = C.beta * C.dt * C.dt, cb = (2 * C.beta - 1) * C.dt * C.dt;
  int iters[kMaxRhs] = {0};
  double relres[kMaxRhs] = {0};
  int solve_iters[4] = {0, 0, 0, 0};
  int sweeps = 0;
  double gres[kMaxRhs] = {0};
  double bn[kMaxRhs];
  int status = DD_OK;
  bool ok = false;  // the refinement residual is below refine_tol for every RHS
  auto nonfinite = [&](const double* v) {
    for (int r = 0; r < nr; ++r)
      if (!std::isfinite(v[r]))
        throw DDError{DD_ERR_NONFINITE, std::string("non-finite entry in the load of right-hand side ") +
                                            std::to_string(r) + " (" + what + ")"};
  };
  const bool refine = C.fp32 && C.opt.refine_max > 0;
  if (tx_done) *tx_done = refine && tx != nullptr;
  // The step as one captured graph once an eager step has shown how many CG
  // iterations and sweeps it needs (first variant, no warm start, a
  // capturable stream, no per-launch timing)
  const bool graph = step && refine && !warm && C.opt.method == 0 && C.nlam > 0 && C.opt.use_graph &&
                     st != nullptr && !C.prof && C.need_iters > 0;
  if (graph) {
    const int I = std::min(C.opt.cg_max_iter, C.need_iters);
    const int S = std::min({C.need_sweeps, C.opt.refine_max, kMaxGraphSweeps});
    Ctx::StepGraph* sg = nullptr;
    for (auto& e : C.step_graphs)
      if (e.g && e.b == b && e.x == x && e.tx == tx && e.sx == sx && e.iters == I && e.sweeps == S) sg = &e;
    if (!sg) {  // the least recently used slot
      sg = &C.step_graphs[0];
      for (auto& e : C.step_graphs)
        if (e.used < sg->used) sg = &e;
      capture_step<T>(C, *sg, b, x, tx, sx, I, S);
    }
    sg->used = ++C.step_clock;
    HIPCHK(hipGraphLaunch(sg->g, st));
    HIPCHK(hipMemcpyAsync(C.h_rs, C.d_rs, sizeof(RefineState), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const RefineState& R = *C.h_rs;
    for (int r = 0; r < nr; ++r) bn[r] = R.bn[r];
    nonfinite(bn);
    int need_it = 0;
    bool capped = false;
    for (int k = 0; k <= S; ++k) {
      if (!R.ran[k]) break;
      if (k > 0) ++sweeps;
      for (int r = 0; r < nr; ++r) {
        iters[r] += R.iters[k][r];
        relres[r] = R.rr0[k][r] > 0 ? std::sqrt(R.rr[k][r] / R.rr0[k][r]) : 0.0;
        need_it = std::max(need_it, R.iters[k][r]);
        if (k < 4) solve_iters[k] = std::max(solve_iters[k], R.iters[k][r]);
      }
      if (R.breakdown[k]) status = DD_ERR_NO_CONVERGENCE;
      if (!R.done[k]) capped = true;  // stopped at I iterations: the refinement carries on
    }
    for (int k = S; k >= 0; --k)
      if (R.checked[k]) {
        for (int r = 0; r < nr; ++r) gres[r] = R.gres[k][r];
        break;
      }
    ok = R.gate[S + 1] != 0;
    C.need_iters = capped ? std::min(C.opt.cg_max_iter, 2 * I) : std::max(need_it, 1);
    // g_r holds b - A x of the last iterate whenever the last check failed
  } else {
    // |b|^2 per RHS before the solve: the reference of the refinement, and a
    // non-finite load is reported instead of being iterated on
    dot_to_host(C, b, b, C.P.nint, bn);
    nonfinite(bn);
    status = dd_solve_once<T>(C, b, x, warm, iters, relres);
    for (int r = 0; r < nr; ++r) solve_iters[0] = std::max(solve_iters[0], iters[r]);
    if (refine) {
      csr_launch(C, st, 1, x, nullptr, nullptr, nullptr, b, ca, cb, C.g_r, tx, nullptr, sx);
      double rn[kMaxRhs];
      dot_to_host(C, C.g_r, C.g_r, C.P.nint, rn);
      ok = true;
      for (int r = 0; r < nr; ++r) {
        gres[r] = bn[r] > 0 ? std::sqrt(rn[r] / bn[r]) : 0.0;
        if (!(gres[r] <= C.opt.refine_tol)) ok = false;
      }
    }
  }
  // eager sweeps: all of them without the graph, those beyond it with it
  while (refine && !ok) {
    if (sweeps >= C.opt.refine_max) {
      status = DD_ERR_NO_CONVERGENCE;
      break;
    }
    int it2[kMaxRhs];
    double rr2[kMaxRhs];
    int s2 = dd_solve_once<T>(C, C.g_r, C.g_t4, nullptr, it2, rr2);
    if (s2 != DD_OK) status = s2;
    for (int r = 0; r < nr; ++r) {
      iters[r] += it2[r];
      if (sweeps + 1 < 4) solve_iters[sweeps + 1] = std::max(solve_iters[sweeps + 1], it2[r]);
    }
    hipLaunchKernelGGL(k_axpy, dim3(nblk(n)), dim3(256), 0, st, n, 1.0, (const double*)C.g_t4, x,
                       (const int*)nullptr);
    ++sweeps;
    csr_launch(C, st, 1, x, nullptr, nullptr, nullptr, b, ca, cb, C.g_r, tx, nullptr, sx);
    double rn[kMaxRhs];
    dot_to_host(C, C.g_r, C.g_r, C.P.nint, rn);
    ok = true;
    for (int r = 0; r < nr; ++r) {
      gres[r] = bn[r] > 0 ? std::sqrt(rn[r] / bn[r]) : 0.0;
      if (!(gres[r] <= C.opt.refine_tol)) ok = false;
    }
  }
  if (step && refine) {
    // what the captured form of the next step must hold
    if (!graph) {
      int m = 1;
      for (int k = 0; k < 4; ++k) m = std::max(m, solve_iters[k]);
      C.need_iters = m;
    }
    C.need_sweeps = sweeps;
  }
  if (stats) {
    std::memset(stats, 0, sizeof(dd_stats));
    for (int r = 0; r < nr; ++r) {
      stats->cg_iters[r] = iters[r];
      stats->cg_relres[r] = relres[r];
      stats->global_relres[r] = gres[r];
    }
    stats->refine_sweeps = sweeps;
    stats->dd_solves = 1 + sweeps;
    for (int k = 0; k < 4; ++k) stats->solve_iters[k] = solve_iters[k];
  }
  return status;
}

// H^{n+1/2} = |e1 - e0|_T^2 / dt^2 + |(e1 + e0)/2|_S^2 per RHS (host out
// [nrhs]) for unknown-major e1, e0, which must not be g_t3, g_t4, g_x or g_r
// (used as scratch).  Synchronises.
static void energy_int(Ctx& C, const double* e1, const double* e0, double* out) {
  const int nr = C.nrhs;
  const int64_t ni = C.P.nint, n = ni * nr;
  hipStream_t st = C.st;
  hipLaunchKernelGGL(k_diff_avg, dim3(nblk(n)), dim3(256), 0, st, n, e1, e0, 1.0 / C.dt, C.g_t3, C.g_t4);
  double a[kMaxRhs], b[kMaxRhs];
  // T dv -> g_x (S dv -> g_r, unused); dv . T dv
  csr_launch(C, st, 3, C.g_t3, nullptr, nullptr, nullptr, nullptr, 0.0, 0.0, C.g_x, C.g_r);
  dot_to_host(C, C.g_t3, C.g_x, ni, a);
  // S av -> g_r (T av -> g_x, unused); av . S av
  csr_launch(C, st, 3, C.g_t4, nullptr, nullptr, nullptr, nullptr, 0.0, 0.0, C.g_x, C.g_r);
  dot_to_host(C, C.g_t4, C.g_r, ni, b);
  for (int r = 0; r < nr; ++r) out[r] = a[r] + b[r];
}

// Diagnostics after a step (DD_DIAG_GAUSS: the charge update with Jint =
// J^{n+1/2} per unknown, and with stats the Gauss-law maxima from tx = T
// e^{n+1} (computed here when have_tx is false); DD_DIAG_ENERGY with stats).
// e1 = e^{n+1}, e0 = e^n per unknown.  Jint and tx must not be g_t3 / g_t4
// / g_x / g_r when the energy is asked for (they are its scratch).
static void step_diagnostics(Ctx& C, const double* Jint, const double* e1, const double* e0, double* tx,
                             bool have_tx, dd_stats* stats) {
  const int nr = C.nrhs;
  hipStream_t st = C.st;
  if (C.opt.diagnostics & DD_DIAG_GAUSS) {
    // q^{n+1} = q^n + dt G^T J^{n+1/2}, with max |G^T T e^{n+1} + q^{n+1}|
    // when the stats are asked for (T e^{n+1} from the last refinement
    // residual, or its own product in the FP64 form)
    if (stats && !have_tx) csr_launch(C, st, 3, e1, nullptr, nullptr, nullptr, nullptr, 0.0, 0.0, tx, C.g_r);
    double* gpart = stats ? C.d_gpart : nullptr;
    // even nrhs: two right-hand sides per lane
    const int lanes = nr % 2 == 0 ? nr / 2 : nr;
    const int vpb = (256 - 256 % lanes) / lanes;
    const unsigned gb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(kGaussBlocks, nblk(C.P.nv, vpb)));
    if (nr % 2 == 0)
      hipLaunchKernelGGL((k_gauss_step_v<2>), dim3(gb), dim3(256), 0, st, (int64_t)C.P.nv, nr, C.d_vptr,
                         C.d_vdof, C.d_nodeint, Jint, C.dt, stats ? (const double*)tx : nullptr, C.d_q, gpart);
    else
      hipLaunchKernelGGL(k_gauss_step, dim3(gb), dim3(256), 0, st, (int64_t)C.P.nv, nr, C.d_vptr,
                         C.d_vdof, C.d_nodeint, Jint, C.dt, stats ? (const double*)tx : nullptr, C.d_q, gpart);
    if (stats) {
      hipLaunchKernelGGL(k_gauss_max, dim3(1), dim3(1024), 0, st, (int)gb, nr, (const double*)C.d_gpart, C.d_gmax);
      HIPCHK(hipMemcpyAsync(C.h_partial, C.d_gmax, sizeof(double) * nr * 2, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      for (int r = 0; r < nr; ++r) {
        stats->gauss_residual[r] = C.h_partial[2 * r];
        stats->charge_max[r] = C.h_partial[2 * r + 1];
      }
    }
  }
}

static void step_energy(Ctx& C, const double* e1, const double* e0, dd_stats* stats) {
  if (stats && (C.opt.diagnostics & DD_DIAG_ENERGY)) energy_int(C, e1, e0, stats->energy);
  if (stats) stats->diagnostics = C.opt.diagnostics & (DD_DIAG_GAUSS | DD_DIAG_ENERGY);
}

template <class T>
static int step_impl(Ctx& C, const double* J1, const double* J0, const double* En, const double* Enm1,
                     double* Enext, dd_stats* stats) {
  const int nr = C.nrhs;
  const int64_t ni = C.P.nint, ne = C.P.ne;
  hipStream_t st = C.st;
  hipLaunchKernelGGL(k_edges_to_int, dim3(nblk(ni, 64)), dim3(256), 0, st, ni, C.d_interior, En, ne, C.g_t1, nr, 1.0);
  hipLaunchKernelGGL(k_edges_to_int, dim3(nblk(ni, 64)), dim3(256), 0, st, ni, C.d_interior, Enm1, ne, C.g_t2, nr, 1.0);
  hipLaunchKernelGGL(k_edges_to_int, dim3(nblk(ni, 64)), dim3(256), 0, st, ni, C.d_interior, J1, ne, C.g_t3, nr, 1.0);
  hipLaunchKernelGGL(k_edges_to_int, dim3(nblk(ni, 64)), dim3(256), 0, st, ni, C.d_interior, J0, ne, C.g_x, nr, 1.0);
  csr_launch(C, st, 0, C.g_t1, C.g_t2, C.g_t3, C.g_x, nullptr, C.beta * C.dt * C.dt, (2 * C.beta - 1) * C.dt * C.dt,
             C.g_b, nullptr);
  // g_t2 (e^{n-1}) is free once the load is assembled: the refinement's last
  // residual leaves T e^{n+1} there for the Gauss check
  const bool gauss = (C.opt.diagnostics & DD_DIAG_GAUSS) != 0;
  bool have_tx = false;
  int status = solve_refined<T>(C, C.g_b, C.g_e, C.opt.warm_start ? &C.warm_fw : nullptr, stats,
                                "J, E_n or E_nm1", gauss ? C.g_t2 : nullptr, &have_tx, true);
  hipLaunchKernelGGL(k_int_to_edges, dim3(nblk(ne, 64)), dim3(256), 0, st, ne, C.d_dof, (const double*)C.g_e,
                     Enext, nr, 0, 1.0);
  // (g_t3 still holds J^{n+1/2} per unknown, converted for the load)
  step_diagnostics(C, C.g_t3, C.g_e, C.g_t1, C.g_t2, have_tx, stats);
  step_energy(C, C.g_e, C.g_t1, stats);
  HIPCHK(hipGetLastError());
  return status;
}

// ---- resident Newmark state ------------------------------------------------------
// The context keeps e^n and e^{n-1} per unknown with their products T e and
// S e, and J^{n-1/2}: a step needs no layout conversion of its inputs but J
// and no sparse product for its load; the accepted iterate's products come
// from the refinement's last residual (or one product without refinement).
static void resident_alloc(Ctx& C) {
  if (C.rs_alloc) return;
  const int64_t n = C.P.nint * C.nrhs;
  for (int k = 0; k < 2; ++k) {
    C.rs_e[k] = dalloc<double>(n, C.owned);
    C.rs_te[k] = dalloc<double>(n, C.owned);
    C.rs_se[k] = dalloc<double>(n, C.owned);
  }
  C.rs_j = dalloc<double>(n, C.owned);
  C.rs_alloc = true;
}

// products of both stored iterates with the current matrices
static void resident_products(Ctx& C) {
  for (int k = 0; k < 2; ++k)
    csr_launch(C, C.st, 3, C.rs_e[k], nullptr, nullptr, nullptr, nullptr, 0.0, 0.0, C.rs_te[k], C.rs_se[k]);
  C.rs_stale = false;
}

static void resident_set(Ctx& C, const double* En, const double* Enm1, const double* Jprev) {
  resident_alloc(C);
  const int nr = C.nrhs;
  const int64_t ni = C.P.nint, ne = C.P.ne, n = ni * nr;
  hipStream_t st = C.st;
  C.rs_p = 0;
  const double* src[3] = {En, Enm1, Jprev};
  double* dst[3] = {C.rs_e[0], C.rs_e[1], C.rs_j};
  for (int k = 0; k < 3; ++k) {
    if (src[k])
      hipLaunchKernelGGL(k_edges_to_int, dim3(nblk(ni, 64)), dim3(256), 0, st, ni, C.d_interior, src[k], ne, dst[k],
                         nr, 1.0);
    else
      hipLaunchKernelGGL(k_zero<double>, dim3(nblk(n)), dim3(256), 0, st, n, dst[k], (const int*)nullptr);
  }
  resident_products(C);
  HIPCHK(hipGetLastError());
}

template <class T>
static int step_resident_impl(Ctx& C, const double* J1, double* Enext, dd_stats* stats) {
  if (!C.rs_alloc) resident_set(C, nullptr, nullptr, nullptr);  // e^0 = e^-1 = 0, J^{-1/2} = 0
  if (C.rs_stale) resident_products(C);
  const int nr = C.nrhs;
  const int64_t ni = C.P.nint, ne = C.P.ne, n = ni * nr;
  hipStream_t st = C.st;
  const int p = C.rs_p, q = 1 - p;  // e^n in slot p; e^{n+1} replaces e^{n-1} in slot q
  hipLaunchKernelGGL(k_edges_to_int, dim3(nblk(ni, 64)), dim3(256), 0, st, ni, C.d_interior, J1, ne, C.g_t3, nr, 1.0);
  hipLaunchKernelGGL(k_newmark_load, dim3(nblk(n)), dim3(256), 0, st, n, (const double*)C.rs_te[p],
                     (const double*)C.rs_se[p], (const double*)C.rs_te[q], (const double*)C.rs_se[q],
                     (const double*)C.g_t3, (const double*)C.rs_j, C.dt, C.beta * C.dt * C.dt,
                     (2 * C.beta - 1) * C.dt * C.dt, C.g_b);
  bool have_tx = false;
  int status = solve_refined<T>(C, C.g_b, C.rs_e[q], C.opt.warm_start ? &C.warm_fw : nullptr, stats, "J",
                                C.rs_te[q], &have_tx, true, C.rs_se[q]);
  if (!have_tx)
    csr_launch(C, st, 3, C.rs_e[q], nullptr, nullptr, nullptr, nullptr, 0.0, 0.0, C.rs_te[q], C.rs_se[q]);
  hipLaunchKernelGGL(k_int_to_edges, dim3(nblk(ne, 64)), dim3(256), 0, st, ne, C.d_dof, (const double*)C.rs_e[q],
                     Enext, nr, 0, 1.0);
  step_diagnostics(C, C.g_t3, C.rs_e[q], C.rs_e[p], C.rs_te[q], true, stats);
  std::swap(C.g_t3, C.rs_j);  // J^{n+1/2} kept; the old buffer becomes scratch
  step_energy(C, C.rs_e[q], C.rs_e[p], stats);
  C.rs_p = q;
  HIPCHK(hipGetLastError());
  return status;
}

template <class T>
static int solve_api_impl(Ctx& C, const double* b, double* x, dd_stats* stats) {
  const int nr = C.nrhs;
  const int64_t ni = C.P.nint, ne = C.P.ne;
  hipStream_t st = C.st;
  hipLaunchKernelGGL(k_edges_to_int, dim3(nblk(ni, 64)), dim3(256), 0, st, ni, C.d_interior, b, ne, C.g_t1, nr,
                     1.0);
  int status = solve_refined<T>(C, C.g_t1, C.g_e, nullptr, stats, "b");
  hipLaunchKernelGGL(k_int_to_edges, dim3(nblk(ne, 64)), dim3(256), 0, st, ne, C.d_dof, (const double*)C.g_e, x,
                     nr, 0, 1.0);
  HIPCHK(hipGetLastError());
  return status;
}

template <class T>
static int adjoint_impl(Ctx& C, const double* ebar_next, double* ebar_n, double* ebar_nm1, double* g_out,
                        const double* E_next, const double* E_n, const double* E_nm1, double* eps_bar,
                        double* Jbar_half, double* Jbar_prev_half, dd_stats* stats) {
  const int nr = C.nrhs;
  const int64_t ni = C.P.nint, ne = C.P.ne;
  hipStream_t st = C.st;
  const int64_t n = ni * nr;
  hipLaunchKernelGGL(k_edges_to_int, dim3(nblk(ni, 64)), dim3(256), 0, st, ni, C.d_interior, ebar_next, ne, C.g_t1, nr,
                     1.0);
  int status = solve_refined<T>(C, C.g_t1, C.g_x, C.opt.warm_start ? &C.warm_adj : nullptr, stats, "ebar_next");
  // B1 g -> g_t2, A g -> g_t3
  csr_launch(C, st, 2, C.g_x, nullptr, nullptr, nullptr, nullptr, C.beta * C.dt * C.dt, (2 * C.beta - 1) * C.dt * C.dt,
             C.g_t2, C.g_t3);
  if (ebar_n)
    hipLaunchKernelGGL(k_int_to_edges, dim3(nblk(ne, 64)), dim3(256), 0, st, ne, C.d_dof, (const double*)C.g_t2,
                       ebar_n, nr, 1, 1.0);
  if (ebar_nm1)
    hipLaunchKernelGGL(k_int_to_edges, dim3(nblk(ne, 64)), dim3(256), 0, st, ne, C.d_dof, (const double*)C.g_t3,
                       ebar_nm1, nr, 1, -1.0);
  if (g_out)
    hipLaunchKernelGGL(k_int_to_edges, dim3(nblk(ne, 64)), dim3(256), 0, st, ne, C.d_dof, (const double*)C.g_x,
                       g_out, nr, 0, 1.0);
  // the load of step n is -dt (J^{n+1/2} - J^{n-1/2})
  if (Jbar_half)
    hipLaunchKernelGGL(k_int_to_edges, dim3(nblk(ne, 64)), dim3(256), 0, st, ne, C.d_dof, (const double*)C.g_x,
                       Jbar_half, nr, 1, -C.dt);
  if (Jbar_prev_half)
    hipLaunchKernelGGL(k_int_to_edges, dim3(nblk(ne, 64)), dim3(256), 0, st, ne, C.d_dof, (const double*)C.g_x,
                       Jbar_prev_half, nr, 1, C.dt);
  if (eps_bar) {
    // acc = e^{n+1} - 2 e^n + e^{n-1} in unknown-major layout
    hipLaunchKernelGGL(k_edges_to_int, dim3(nblk(ni, 64)), dim3(256), 0, st, ni, C.d_interior, E_next, ne, C.g_t2, nr,
                       1.0);
    hipLaunchKernelGGL(k_edges_to_int, dim3(nblk(ni, 64)), dim3(256), 0, st, ni, C.d_interior, E_n, ne, C.g_t3, nr,
                       1.0);
    if (E_nm1)
      hipLaunchKernelGGL(k_edges_to_int, dim3(nblk(ni, 64)), dim3(256), 0, st, ni, C.d_interior, E_nm1, ne, C.g_t4,
                         nr, 1.0);
    hipLaunchKernelGGL(k_second_diff, dim3(nblk(n)), dim3(256), 0, st, n, (const double*)C.g_t2,
                       (const double*)C.g_t3, (const double*)(E_nm1 ? C.g_t4 : nullptr), C.g_t2);
    hipLaunchKernelGGL(k_eps_bar, dim3(nblk(C.P.nt)), dim3(256), 0, st, (int64_t)C.P.nt, C.d_tdof, C.d_Te,
                       (const double*)C.g_x, (const double*)C.g_t2, nr, eps_bar);
  }
  HIPCHK(hipGetLastError());
  return status;
}

// ---------------------------------------------------------------------------
// autotuner of the work-list shapes
// ---------------------------------------------------------------------------
// Rebuild the work lists of the classes in `which` (1: interface blocks and
// corner rows, 2: coarse, 4: full r-blocks) with the current tuning.  The
// tile lists (mlist) do not depend on the chunking and are kept.  The
// captured CG graph holds the old lists, so it is dropped (recaptured on the
// next solve).
template <class T>
static void rebuild_lists(Ctx& C, int which) {
  auto remake = [&](Items& it, const std::vector<MvItem>& blk, int chunk, bool grouped, int bucket) {
    int32_t* ml = it.mlist;
    it.mlist = nullptr;
    release_items(C, it);
    it = make_items(C, blk, chunk, grouped, bucket);
    it.mlist = ml;
  };
  HIPCHK(hipStreamSynchronize(C.st));
  drop_graphs(C);
  if (which & 1) {
    remake(C.corner_N, C.blk_corner_N, C.tuning.chunk, false, 1);
    remake(C.corner_T, C.blk_corner_T, C.tuning.chunk, false, 1);
  }
  if ((which & 2) && C.coarse_lists) {
    remake(C.co_N, C.blk_co_N, C.tuning.coarse_chunk, false, 1);
    remake(C.co_T, C.blk_co_T, C.tuning.coarse_chunk, false, 1);
  }
  if ((which & 4) && C.full_N.d) build_full_items<T>(C);
  if ((which & 8) && C.sym.pw != sym_width(C)) make_sym_list(C, sym_width(C), sizeof(T));
  ensure_partial<T>(C);
}

// Cache key of a tuning: device, precision, RHS count and a hash of the
// subdomain tile shapes and the nonzero-tile pattern of the full lists.
static std::string tune_key(const Ctx& C) {
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, C.device));
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    for (int b = 0; b < 8; ++b) {
      h ^= (v >> (8 * b)) & 0xff;
      h *= 1099511628211ull;
    }
  };
  for (const SubDev& q : C.subs_h) {
    mix((uint64_t)q.kI);
    mix((uint64_t)q.kG);
    mix((uint64_t)q.kC);
  }
  for (uint8_t b : C.full_pattern) mix(b);
  char buf[256];
  std::snprintf(buf, sizeof buf, "%s/%s/nrhs%d/nsub%d/%016llx", prop.gcnArchName, C.fp32 ? "fp32" : "fp64",
                C.nrhs, C.nsub, (unsigned long long)h);
  return buf;
}

// The integer value of "name": in one line of the cache, or -1.
static long json_int(const std::string& line, const char* name) {
  const std::string k = std::string("\"") + name + "\":";
  size_t p = line.find(k);
  if (p == std::string::npos) return -1;
  return std::strtol(line.c_str() + p + k.size(), nullptr, 10);
}

// Look the key up in the cache (JSON lines: one object per tuning).
static bool tune_cache_read(const std::string& path, const std::string& key, Tuning& t) {
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  char buf[4096];
  bool found = false;
  const std::string kq = "\"key\": \"" + key + "\"";
  while (std::fgets(buf, sizeof buf, f)) {
    std::string line(buf);
    if (line.find(kq) == std::string::npos) continue;
    Tuning c;
    long v[4] = {json_int(line, "chunk"), json_int(line, "coarse_chunk"), json_int(line, "full_chunk"),
                 json_int(line, "full_bucket")};
    const long fp = json_int(line, "full_persist");
    const long fpair = json_int(line, "full_pair");
    if (v[0] < 1 || v[1] < 1 || v[2] < 1 || v[3] < 1 || v[0] > 4096 || v[1] > 4096 || v[2] > 4096 ||
        v[3] > (1 << 20))
      continue;
    c.chunk = (int)v[0];
    c.coarse_chunk = (int)v[1];
    c.full_chunk = (int)v[2];
    c.full_bucket = (int)v[3];
    // a persistent grid must be a multiple of 8 workgroups (absent or bad: none)
    c.full_persist = (fp > 0 && fp % 8 == 0 && fp <= (1L << 24)) ? (int)fp : 0;
    c.full_pair = (fpair == 1 || fpair == 2) ? (int)fpair : 0;
    c.full_quarter = json_int(line, "full_quarter") == 0 ? 0 : 1;
    const long sp = json_int(line, "sym_persist");
    c.sym_persist = (sp > 0 && sp % 8 == 0 && sp <= (1L << 24)) ? (int)sp : 0;
    c.sym_pw = json_int(line, "sym_pw") == 2 ? 2 : 0;
    t = c;
    found = true;  // the last entry for a key wins
  }
  std::fclose(f);
  return found;
}

static void tune_cache_append(const std::string& path, const std::string& key, const Tuning& t,
                              const dd_tuning& r) {
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) throw DDError{DD_ERR_ARG, "cannot open the tuning cache " + path + " for writing"};
  std::fprintf(f,
               "{\"key\": \"%s\", \"chunk\": %d, \"coarse_chunk\": %d, \"full_chunk\": %d, "
               "\"full_bucket\": %d, \"full_persist\": %d, \"full_pair\": %d, \"full_quarter\": %d, "
               "\"sym_pw\": %d, \"sym_persist\": %d, \"local_ms\": %.5f, \"local_ms_default\": %.5f, "
               "\"full_ms\": %.5f, "
               "\"full_ms_default\": %.5f, "
               "\"coarse_ms\": %.5f, \"coarse_ms_default\": %.5f, \"trailing_ms\": %.5f, "
               "\"trailing_ms_default\": %.5f}\n",
               key.c_str(), t.chunk, t.coarse_chunk, t.full_chunk, t.full_bucket, t.full_persist, t.full_pair,
               t.full_quarter, t.sym_pw, t.sym_persist, r.local_ms, r.local_ms_default, r.full_ms,
               r.full_ms_default, r.coarse_ms, r.coarse_ms_default, r.trailing_ms, r.trailing_ms_default);
  std::fclose(f);
}

// Time every candidate shape of each product class (the products of one DD
// solve, on zero vectors: the time does not depend on the values), keep the
// fastest, and leave the lists built with it.  Per class: the median of 5
// timed repetitions after a warm-up, with HIP events on the context stream.
template <class T>
static void autotune_impl(Ctx& C, dd_tuning* out) {
  hipStream_t st = C.st;
  const T one = 1, mone = -1;
  const size_t vb = (size_t)std::max<int64_t>(1, C.rows_total) * C.nrhs * sizeof(T);
  for (int i = 0; i < 8; ++i) HIPCHK(hipMemsetAsync(C.X[i], 0, vb, st));
  hipEvent_t ev[6];
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  struct Guard {
    hipEvent_t* e;
    ~Guard() {
      for (int i = 0; i < 6; ++i) (void)hipEventDestroy(e[i]);
    }
  } guard{ev};
  auto timed = [&](auto&& fn) -> double {
    fn();
    float ms[5];
    for (int r = 0; r < 5; ++r) {
      HIPCHK(hipEventRecord(ev[0], st));
      fn();
      HIPCHK(hipEventRecord(ev[1], st));
      HIPCHK(hipEventSynchronize(ev[1]));
      HIPCHK(hipEventElapsedTime(&ms[r], ev[0], ev[1]));
    }
    std::sort(ms, ms + 5);
    return ms[2];
  };
  void** X = C.X;
  auto full = [&] {
    mv<T>(C, C.full_N, false, X[0], X[1], nullptr, one);
    mv<T>(C, C.cross_N, false, X[1], X[2], X[0], mone, nullptr, X[0], mone);
    mv<T>(C, C.cross_T, true, X[5], X[2], X[1], mone);
    mv<T>(C, C.full_T, true, X[2], X[5], nullptr, one);
  };
  auto coarse = [&] { coarse_solve<T>(C, X[6], X[7], X[5], nullptr); };
  // (the corner-coupling passes; the result fields keep their names)
  auto trailing = [&] {
    mv<T>(C, C.corner_N, false, X[5], X[6], nullptr, one);
    mv<T>(C, C.corner_T, true, X[6], X[8], nullptr, one);
  };
  const bool prof = C.prof;
  C.prof = false;
  Tuning best = C.tuning;
  dd_tuning r{};
  // full passes: chunk length x placement bucket
  if (C.full_N.d) {
    r.full_ms_default = r.full_ms = timed(full);
    // (bucket 1 << 20: one bucket, so each XCD takes its subdomains one
    // after the other in the given order, rows in order)
    for (int fc : {48, 64, 96, 128, 192})
      for (int b : {1, 4, 8, 16, 1 << 20}) {
        C.tuning.full_chunk = fc;
        C.tuning.full_bucket = b;
        rebuild_lists<T>(C, 4);
        const double t = timed(full);
        if (t < r.full_ms) {
          r.full_ms = t;
          best.full_chunk = fc;
          best.full_bucket = b;
        }
      }
  }
  C.tuning = best;
  rebuild_lists<T>(C, 4);
  // reading whole tiles, zero quarters included
  if (C.full_N.d) {
    C.tuning.full_quarter = 0;
    rebuild_lists<T>(C, 4);
    const double t = timed(full);
    if (t < r.full_ms) {
      r.full_ms = t;
      best.full_quarter = 0;
    }
    C.tuning = best;
    rebuild_lists<T>(C, 4);
  }
  // row pairs (two output rows per wave), then a persistent grid
  if (C.full_N.d && C.nrhs > 8) {
    for (int fc : {32, 48, 64, 96})
      for (int b : {best.full_bucket, 1 << 20}) {
        C.tuning.full_pair = 1;
        C.tuning.full_chunk = fc;
        C.tuning.full_bucket = b;
        rebuild_lists<T>(C, 4);
        const double t = timed(full);
        if (t < r.full_ms) {
          r.full_ms = t;
          best.full_pair = 1;
          best.full_chunk = fc;
          best.full_bucket = b;
        }
      }
    // eight rows per workgroup (not split; the chunk does not apply)
    for (int b : {best.full_bucket, 1 << 20}) {
      C.tuning.full_pair = 2;
      C.tuning.full_bucket = b;
      rebuild_lists<T>(C, 4);
      const double t = timed(full);
      if (t < r.full_ms) {
        r.full_ms = t;
        best.full_pair = 2;
        best.full_bucket = b;
      }
    }
    C.tuning = best;
    rebuild_lists<T>(C, 4);
  }
  if (C.full_N.d) {
    for (int pg : {1024, 2048, 4096, 8192}) {
      C.tuning.full_persist = pg;
      const double t = timed(full);
      if (t < r.full_ms) {
        r.full_ms = t;
        best.full_persist = pg;
      }
    }
    C.tuning = best;
  }
  if (C.Kc > 0 && C.coarse_lists) {
    r.coarse_ms_default = r.coarse_ms = timed(coarse);
    for (int cc : {8, 12, 16, 24, 32, 48}) {
      C.tuning.coarse_chunk = cc;
      rebuild_lists<T>(C, 2);
      const double t = timed(coarse);
      if (t < r.coarse_ms) {
        r.coarse_ms = t;
        best.coarse_chunk = cc;
      }
    }
  }
  C.tuning = best;
  rebuild_lists<T>(C, 2);
  r.trailing_ms_default = r.trailing_ms = timed(trailing);
  for (int ch : {16, 24, 32, 48, 64}) {
    C.tuning.chunk = ch;
    rebuild_lists<T>(C, 1);
    const double t = timed(trailing);
    if (t < r.trailing_ms) {
      r.trailing_ms = t;
      best.chunk = ch;
    }
  }
  C.tuning = best;
  rebuild_lists<T>(C, 1);
  // the local response of one interface-operator application: the
  // symmetric product on the side stream beside the corner and coarse chain
  // (a persistent grid of the symmetric product leaves the chain free slots)
  if (C.sym.n > 0 && C.Kc > 0) {
    auto local = [&] { apply_local<T>(C, nullptr); };
    r.local_ms_default = r.local_ms = timed(local);
    if (C.fp32) {
      // panel width 2: half the accumulators per wave (more waves per SIMD),
      // twice the partial slots
      C.tuning.sym_pw = 2;
      rebuild_lists<T>(C, 8);
      const double t = timed(local);
      if (t < r.local_ms) {
        r.local_ms = t;
        best.sym_pw = 2;
      }
      C.tuning = best;
      rebuild_lists<T>(C, 8);
    }
    for (int pg : {256, 512, 768, 1024, 1536, 2048}) {
      C.tuning.sym_persist = pg;
      const double t = timed(local);
      if (t < r.local_ms) {
        r.local_ms = t;
        best.sym_persist = pg;
      }
    }
    C.tuning = best;
  }
  C.prof = prof;
  r.chunk = best.chunk;
  r.coarse_chunk = best.coarse_chunk;
  r.full_chunk = best.full_chunk;
  r.full_bucket = best.full_bucket;
  r.full_persist = best.full_persist;
  r.full_pair = best.full_pair;
  r.full_quarter = best.full_quarter;
  r.sym_persist = best.sym_persist;
  r.sym_pw = best.sym_pw;
  if (out) *out = r;
}

// dd_autotune: cached tuning if the cache has the key, else a timed search
// (appended to the cache when one is given).
template <class T>
static void autotune(Ctx& C, const char* cache, dd_tuning* out) {
  const std::string key = tune_key(C);
  dd_tuning r{};
  Tuning t;
  if (cache && *cache && tune_cache_read(cache, key, t)) {
    C.tuning = t;
    rebuild_lists<T>(C, 15);
    r.chunk = t.chunk;
    r.coarse_chunk = t.coarse_chunk;
    r.full_chunk = t.full_chunk;
    r.full_bucket = t.full_bucket;
    r.full_persist = t.full_persist;
    r.full_pair = t.full_pair;
    r.full_quarter = t.full_quarter;
    r.sym_persist = t.sym_persist;
    r.sym_pw = t.sym_pw;
    r.from_cache = 1;
  } else {
    autotune_impl<T>(C, &r);
    if (cache && *cache) tune_cache_append(cache, key, C.tuning, r);
  }
  C.tune_applied = true;
  if (out) *out = r;
}

}  // namespace ddfem

using namespace ddfem;

// Scratch of dd_pic_sort_noalloc: the per-cell counts, then cursors [cells + 1],
// followed by the scan's chunk totals, in one file-scope device array of fixed
// size (16.0 MiB), so that the call allocates nothing.  Each device holds its
// own copy for the life of the process; host code uses only the addresses
// resolved per device by resolve_scratch, never the symbol itself.
constexpr int64_t kNoAllocMaxCells = int64_t(1) << 22;
constexpr int64_t kNoAllocChunks = (kNoAllocMaxCells + 1 + kScanBlock - 1) / kScanBlock;
static __device__ __align__(256) int32_t scratch[kNoAllocMaxCells + 1 + kNoAllocChunks];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static int32_t* g_scratch_ptr[kMaxDevices] = {};

// Device address of scratch on device dev (current), resolved once per device.
static void resolve_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) throw DDError{DD_ERR_HIP, "device id out of range"};
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return;
  void* p = nullptr;
  HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw DDError{DD_ERR_HIP, "no device address for the static scratch"};
  g_scratch_ptr[dev] = (int32_t*)p;
}

static int32_t* scratch_of(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (dev >= 0 && dev < kMaxDevices) ? g_scratch_ptr[dev] : nullptr;
}

// ===========================================================================
// C ABI
// ===========================================================================
// ---- Robin variant: side maps, interface face masses, Robin terms ----------------
// Tangential mass of the three edges (01, 02, 12) of a triangle p0 p1 p2 with
// vertices in ascending global id: int_F (n x W_a).(n x W_b) dS, where the
// tangential trace of a Whitney function on F is the triangle's own Whitney
// function mu_i grad mu_j - mu_j grad mu_i, and int_F mu_a mu_b = A (1 + d_ab) / 12.
static void face_tangential_mass(const double* p0, const double* p1, const double* p2, double M[3][3]) {
  double e1[3], e2[3];
  for (int c = 0; c < 3; ++c) {
    e1[c] = p1[c] - p0[c];
    e2[c] = p2[c] - p0[c];
  }
  const double a = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
  const double b = e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2];
  const double d = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
  const double det = a * d - b * b;  // |e1 x e2|^2
  double g[3][3];
  for (int c = 0; c < 3; ++c) {
    g[1][c] = (d * e1[c] - b * e2[c]) / det;
    g[2][c] = (a * e2[c] - b * e1[c]) / det;
    g[0][c] = -(g[1][c] + g[2][c]);
  }
  const double area = 0.5 * std::sqrt(det);
  auto gg = [&](int i, int j) { return g[i][0] * g[j][0] + g[i][1] * g[j][1] + g[i][2] * g[j][2]; };
  auto mm = [](int i, int j) { return (i == j ? 2.0 : 1.0) / 12.0; };
  const int LE[3][2] = {{0, 1}, {0, 2}, {1, 2}};
  for (int A = 0; A < 3; ++A)
    for (int B = 0; B < 3; ++B) {
      const int i = LE[A][0], j = LE[A][1], k = LE[B][0], l = LE[B][1];
      M[A][B] = area * (mm(i, k) * gg(j, l) - mm(i, l) * gg(j, k) - mm(j, k) * gg(i, l) + mm(j, l) * gg(i, k));
    }
}

static void build_dp2(Ctx& C, const double* coords, const double* eps, const double* mu) {
  const Plan& P = C.P;
  hipStream_t st = C.st;
  const int nsub = C.nsub;
  const int nr = C.nrhs;
  // side index = position in the interface-row list (d_grow)
  std::vector<int64_t> gbase(nsub + 1, 0);
  for (int s = 0; s < nsub; ++s) gbase[s + 1] = gbase[s] + (int64_t)(P.subs[s].kr() - P.subs[s].kI) * NB;
  const int64_t ns = gbase[nsub];
  if (ns != C.n_grow) throw DDError{DD_ERR_STATE, "interface row count mismatch"};
  if (ns > INT32_MAX / 2) throw DDError{DD_ERR_ARG, "too many interface rows for the Robin variant"};
  std::vector<int32_t> code2(ns, -1), partner2(ns, -1);
  const int64_t nl = P.nlambda();
  std::vector<int32_t> lam_of_dof(P.nint, -1);
  std::vector<int64_t> side0(nl), side1(nl);
  for (int64_t l = 0; l < nl; ++l) {
    const int s0 = P.lam_s0[l], s1 = P.lam_s1[l];
    side0[l] = gbase[s0] + (P.lam_p0[l] - P.subs[s0].nI);
    side1[l] = gbase[s1] + (P.lam_p1[l] - P.subs[s1].nI);
    code2[side0[l]] = (int32_t)(side0[l] << 1);
    code2[side1[l]] = (int32_t)(side1[l] << 1);
    partner2[side0[l]] = (int32_t)side1[l];
    partner2[side1[l]] = (int32_t)side0[l];
    lam_of_dof[P.lam_dof[l]] = (int32_t)l;
  }
  auto side_in = [&](int64_t l, int s) { return P.lam_s0[l] == s ? side0[l] : side1[l]; };
  auto row_in = [&](int64_t l, int s) {
    return P.lam_s0[l] == s ? P.padded_row(s, P.lam_p0[l]) : P.padded_row(s, P.lam_p1[l]);
  };
  // alpha: half the sum of the mass and curl-curl scales of an edge unknown,
  // eps h and beta dt^2 / (mu h), h the mean edge length
  double hsum = 0.0;
  for (int64_t e = 0; e < P.ne; ++e) {
    const double* a = coords + 3 * (int64_t)P.edges[2 * e];
    const double* b = coords + 3 * (int64_t)P.edges[2 * e + 1];
    hsum += std::sqrt((a[0] - b[0]) * (a[0] - b[0]) + (a[1] - b[1]) * (a[1] - b[1]) + (a[2] - b[2]) * (a[2] - b[2]));
  }
  const double h = hsum / std::max<int64_t>(1, P.ne);
  double es = 0.0, ms = 0.0;
  for (int64_t t = 0; t < P.nt; ++t) {
    es += eps[t];
    ms += mu ? mu[t] : 1.0;
  }
  es /= std::max<int64_t>(1, P.nt);
  ms /= std::max<int64_t>(1, P.nt);
  C.robin_alpha = C.opt.robin_alpha > 0 ? C.opt.robin_alpha : 0.5 * (es * h + C.beta * C.dt * C.dt / (ms * h));
  // interface faces: R entries (side space) and Robin terms of both local blocks
  std::vector<int32_t> nbr;
  std::string msg;
  if (face_neighbors(P, nbr, msg) != 0) throw DDError{DD_ERR_MESH, msg};
  std::vector<std::tuple<int64_t, int64_t, double>> R;
  std::vector<std::pair<int64_t, double>> add;
  const int LE6[4][4] = {{-1, 0, 1, 2}, {0, -1, 3, 4}, {1, 3, -1, 5}, {2, 4, 5, -1}};
  for (int64_t t = 0; t < P.nt; ++t)
    for (int k = 0; k < 4; ++k) {
      const int64_t u = nbr[4 * t + k];
      if (u < 0 || u < t) continue;
      const int s = P.part[t], j = P.part[u];
      if (s == j) continue;
      int L[3], m = 0;
      for (int i = 0; i < 4; ++i)
        if (i != k) L[m++] = i;
      double M[3][3];
      face_tangential_mass(coords + 3 * (int64_t)P.tsort[4 * t + L[0]], coords + 3 * (int64_t)P.tsort[4 * t + L[1]],
                           coords + 3 * (int64_t)P.tsort[4 * t + L[2]], M);
      const int FE[3][2] = {{0, 1}, {0, 2}, {1, 2}};
      int64_t lam[3];
      for (int a = 0; a < 3; ++a) {
        const int32_t d = P.dof[P.tet_edges[6 * t + LE6[L[FE[a][0]]][L[FE[a][1]]]]];
        lam[a] = d >= 0 ? lam_of_dof[d] : -1;
      }
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          if (lam[a] < 0 || lam[b] < 0) continue;
          const double v = M[a][b];
          R.emplace_back(side_in(lam[a], s), side_in(lam[b], j), 2.0 * C.robin_alpha * v);
          R.emplace_back(side_in(lam[a], j), side_in(lam[b], s), 2.0 * C.robin_alpha * v);
          for (int q : {s, j}) {
            const int32_t ra = row_in(lam[a], q), rb = row_in(lam[b], q);
            if (ra < rb) continue;
            const SubDev& qd = C.subs_h[q];
            const int64_t ti = qd.tile_off + (int64_t)(ra / NB) * (ra / NB + 1) / 2 + rb / NB;
            add.emplace_back(ti * kTile + (ra % NB) * NB + (rb % NB), v);
          }
        }
    }
  std::sort(R.begin(), R.end());
  std::vector<int64_t> rrp(ns + 1, 0);
  std::vector<int32_t> rci;
  std::vector<double> rval;
  for (size_t i = 0; i < R.size();) {
    size_t k = i;
    double v = 0.0;
    while (k < R.size() && std::get<0>(R[k]) == std::get<0>(R[i]) && std::get<1>(R[k]) == std::get<1>(R[i]))
      v += std::get<2>(R[k++]);
    rrp[std::get<0>(R[i]) + 1]++;
    rci.push_back((int32_t)std::get<1>(R[i]));
    rval.push_back(v);
    i = k;
  }
  for (int64_t i = 0; i < ns; ++i) rrp[i + 1] += rrp[i];
  std::sort(add.begin(), add.end());
  std::vector<int64_t> apos;
  std::vector<double> aval;
  for (size_t i = 0; i < add.size();) {
    size_t k = i;
    double v = 0.0;
    while (k < add.size() && add[k].first == add[i].first) v += add[k++].second;
    apos.push_back(add[i].first);
    aval.push_back(v);
    i = k;
  }
  C.d_code2 = upload(code2, C.owned, st);
  C.d_partner2 = upload(partner2, C.owned, st);
  C.d_rrp = upload(rrp, C.owned, st);
  {
    // the local row of every column's side (the side order is that of d_grow)
    std::vector<int64_t> row_of(ns);
    for (int s = 0; s < nsub; ++s)
      for (int64_t x = gbase[s]; x < gbase[s + 1]; ++x)
        row_of[x] = C.subs_h[s].row_off + (int64_t)P.subs[s].kI * NB + (x - gbase[s]);
    std::vector<int64_t> rrow(rci.size());
    for (size_t j = 0; j < rci.size(); ++j) rrow[j] = row_of[rci[j]];
    C.d_rrow = upload(rrow, C.owned, st);
  }
  C.d_rval = upload(rval, C.owned, st);
  C.n_radd = (int64_t)apos.size();
  C.d_radd_pos = upload(apos, C.owned, st);
  C.d_radd_val = upload(aval, C.owned, st);
  const int64_t nv = ns * nr;
  C.d_gmV = dalloc<double>((size_t)(kGmresRestart + 1) * nv, C.owned);
  C.d_gm_rhs = dalloc<double>(nv, C.owned);
  C.d_lam2 = dalloc<double>(nv, C.owned);
  C.d_gm_partial = dalloc<double>((size_t)(kGmresRestart + 1) * kDotBlocks * kMaxRhs, C.owned);
  C.d_gm_h = dalloc<double>((size_t)(kGmresRestart + 1) * kMaxRhs, C.owned);
  C.d_gm_tot = dalloc<double>((size_t)(kGmresRestart + 1) * kMaxRhs, C.owned);
  C.d_gm_y = dalloc<double>((size_t)kGmresRestart * kMaxRhs, C.owned);
  C.d_gm_wpart = dalloc<double>((size_t)kDotBlocks * kMaxRhs, C.owned);  // |rhs|^2, |r0|^2 block shares
  C.d_gm_H = dalloc<double>((size_t)nr * kGmresRestart * (kGmresRestart + 1), C.owned);
  C.d_gm_cs = dalloc<double>((size_t)nr * kGmresRestart, C.owned);
  C.d_gm_sn = dalloc<double>((size_t)nr * kGmresRestart, C.owned);
  C.d_gm_g = dalloc<double>((size_t)nr * (kGmresRestart + 1), C.owned);
  C.d_gm_st = dalloc<GmState>(1, C.owned);
  HIPCHK(hipHostMalloc((void**)&C.h_gm_st, sizeof(GmState), hipHostMallocDefault));
}

// ---- particle tables (built on the first particle call) --------------------------
static void pic_prepare(Ctx& C) {
  if (C.d_pic_geo) return;
  const Plan& P = C.P;
  std::vector<int32_t> nbr;
  std::string msg;
  if (face_neighbors(P, nbr, msg) != 0) throw DDError{DD_ERR_MESH, msg};
  C.d_pic_nbr = upload(nbr, C.owned, C.st);
  C.d_pic_tedge = upload(P.tet_edges, C.owned, C.st);
  C.d_pic_cnt = dalloc<unsigned long long>(kPicCounters, C.owned);
  HIPCHK(hipMemsetAsync(C.d_pic_cnt, 0, kPicCounters * sizeof(unsigned long long), C.st));
  C.d_pic_count = dalloc<int32_t>((size_t)P.nt + 1, C.owned);
  C.d_pic_bsum = dalloc<int32_t>((size_t)(P.nt + 1 + kScanBlock - 1) / kScanBlock, C.owned);
  double* geo = dalloc<double>((size_t)P.nt * 12, C.owned);
  hipLaunchKernelGGL(k_tet_geo, dim3(nblk(P.nt)), dim3(256), 0, C.st, (int64_t)P.nt, C.d_coords, C.d_tsort, geo);
  HIPCHK(hipGetLastError());
  C.d_pic_geo = geo;
}

// ---- mixed E/B step (Sec. II-B-1, trapezoid rule) ---------------------------------
static void mixed_prepare(Ctx& C) {
  if (C.d_tet_faces) return;
  pic_prepare(C);
  const Plan& P = C.P;
  struct Face {
    int32_t a, b, c;
    int64_t slot;  // 4t + k (face opposite local vertex k)
  };
  std::vector<Face> f((size_t)P.nt * 4);
  for (int64_t t = 0; t < P.nt; ++t)
    for (int k = 0; k < 4; ++k) {
      const int32_t* v = &P.tsort[4 * t];
      f[4 * t + k] = Face{v[kLocFaces[k][0]], v[kLocFaces[k][1]], v[kLocFaces[k][2]], 4 * t + k};
    }
  std::sort(f.begin(), f.end(), [](const Face& x, const Face& y) {
    if (x.a != y.a) return x.a < y.a;
    if (x.b != y.b) return x.b < y.b;
    if (x.c != y.c) return x.c < y.c;
    return x.slot < y.slot;
  });
  std::vector<int32_t> tet_faces((size_t)P.nt * 4), face_edges;
  C.faces_h.clear();
  const int LE6[4][4] = {{-1, 0, 1, 2}, {0, -1, 3, 4}, {1, 3, -1, 5}, {2, 4, 5, -1}};
  for (size_t i = 0; i < f.size();) {
    size_t j = i;
    const int64_t id = (int64_t)C.faces_h.size() / 3;
    if (id > INT32_MAX) throw DDError{DD_ERR_ARG, "too many faces"};
    while (j < f.size() && f[j].a == f[i].a && f[j].b == f[i].b && f[j].c == f[i].c) tet_faces[f[j++].slot] = (int32_t)id;
    C.faces_h.insert(C.faces_h.end(), {f[i].a, f[i].b, f[i].c});
    // edges (ab, bc, ac) from the first tetrahedron holding the face
    const int64_t t = f[i].slot / 4;
    const int k = (int)(f[i].slot % 4);
    const int* L = kLocFaces[k];
    face_edges.push_back(P.tet_edges[6 * t + LE6[L[0]][L[1]]]);
    face_edges.push_back(P.tet_edges[6 * t + LE6[L[1]][L[2]]]);
    face_edges.push_back(P.tet_edges[6 * t + LE6[L[0]][L[2]]]);
    i = j;
  }
  C.n_faces = (int64_t)C.faces_h.size() / 3;
  // unknown d <- (tet, local edge) entries, tetrahedra ascending
  std::vector<int64_t> ptr(P.nint + 1, 0);
  for (int64_t i = 0; i < P.nt * 6; ++i) {
    const int32_t d = P.dof[P.tet_edges[i]];
    if (d >= 0) ptr[d + 1]++;
  }
  for (int64_t d = 0; d < P.nint; ++d) ptr[d + 1] += ptr[d];
  std::vector<int32_t> list(ptr[P.nint]);
  std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
  if (P.nt * 6 > INT32_MAX) throw DDError{DD_ERR_ARG, "too many tetrahedra for the mixed step"};
  for (int64_t i = 0; i < P.nt * 6; ++i) {
    const int32_t d = P.dof[P.tet_edges[i]];
    if (d >= 0) list[fill[d]++] = (int32_t)i;
  }
  C.d_tet_faces = upload(tet_faces, C.owned, C.st);
  C.d_face_edges = upload(face_edges, C.owned, C.st);
  C.d_e6ptr = upload(ptr, C.owned, C.st);
  C.d_e6list = upload(list, C.owned, C.st);
  C.d_buf6 = dalloc<double>((size_t)P.nt * 6 * C.nrhs, C.owned);
  C.d_bt = dalloc<double>((size_t)C.n_faces * C.nrhs, C.owned);
}

template <class T>
static int mixed_step_impl(Ctx& C, const double* J1, const double* En, const double* Bn, double* Enext,
                           double* Bnext, dd_stats* stats) {
  const int nr = C.nrhs;
  const int64_t ni = C.P.nint, ne = C.P.ne, nf = C.n_faces, nt = C.P.nt;
  hipStream_t st = C.st;
  const int64_t n = ni * nr;
  hipLaunchKernelGGL(k_edges_to_int, dim3(nblk(ni, 64)), dim3(256), 0, st, ni, C.d_interior, En, ne, C.g_t1, nr, 1.0);
  hipLaunchKernelGGL(k_edges_to_int, dim3(nblk(ni, 64)), dim3(256), 0, st, ni, C.d_interior, J1, ne, C.g_t3, nr, 1.0);
  // T e -> g_t2, S e -> g_x
  csr_launch(C, st, 3, C.g_t1, nullptr, nullptr, nullptr, nullptr, 0.0, 0.0, C.g_t2, C.g_x);
  // C^T M b -> g_e (a free buffer until the solve)
  hipLaunchKernelGGL(k_rhs_major_to_item, dim3(nblk(nf * nr)), dim3(256), 0, st, nf, nr, Bn, C.d_bt);
  hipLaunchKernelGGL(k_curlT_face_mass, dim3(nblk(nt * nr)), dim3(256), 0, st, nt, nr, (const double*)C.d_bt,
                     (const int32_t*)C.d_tet_faces, (const double*)C.d_pic_geo, (const double*)C.d_mu, C.d_buf6);
  hipLaunchKernelGGL(k_pull_edge6, dim3(nblk(n)), dim3(256), 0, st, ni, nr, (const int64_t*)C.d_e6ptr,
                     (const int32_t*)C.d_e6list, (const double*)C.d_buf6, C.g_e);
  hipLaunchKernelGGL(k_mixed_rhs, dim3(nblk(n)), dim3(256), 0, st, n, (const double*)C.g_t2, (const double*)C.g_x,
                     (const double*)C.g_e, (const double*)C.g_t3, C.dt, C.g_b);
  int status = solve_refined<T>(C, C.g_b, C.g_e, nullptr, stats);
  hipLaunchKernelGGL(k_int_to_edges, dim3(nblk(ne, 64)), dim3(256), 0, st, ne, C.d_dof, (const double*)C.g_e,
                     Enext, nr, 0, 1.0);
  hipLaunchKernelGGL(k_face_update, dim3(nblk(nf * nr)), dim3(256), 0, st, nf, nr, ne,
                     (const int32_t*)C.d_face_edges, En, (const double*)Enext, Bn, Bnext, 0.5 * C.dt);
  HIPCHK(hipGetLastError());
  return status;
}

#define API_BEGIN try {
#define API_END                                 \
  }                                             \
  catch (const DDError& e) {                    \
    g_err = e.msg;                              \
    return e.code;                              \
  }                                             \
  catch (const std::bad_alloc&) {               \
    g_err = "host allocation failed";           \
    return DD_ERR_OOM;                          \
  }                                             \
  catch (const std::exception& e) {             \
    g_err = e.what();                           \
    return DD_ERR_ARG;                          \
  }

extern "C" {

void dd_default_options(dd_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = DD_FP64;
  o->nrhs = 1;
  o->cg_tol = 1e-10;
  o->cg_max_iter = 500;
  o->refine_tol = 1e-12;
  o->refine_max = 10;
  o->warm_start = 0;  // with the preconditioner a warm start saves no iteration
  o->use_graph = 0;
  o->check_every = 4;
  o->stream = nullptr;
  o->precond = 1;
  o->method = 0;
  o->robin_alpha = 0.0;
  o->diagnostics = 0;
}

const char* dd_last_error(void) { return g_err.c_str(); }

static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

int dd_setup(void** out, const dd_mesh* mesh, const int32_t* partition, const double* eps, const double* mu,
             double dt, double beta, const dd_options* opt) {
  g_err.clear();
  if (!out) {
    g_err = "out is NULL";
    return DD_ERR_ARG;
  }
  *out = nullptr;
  Ctx* C = nullptr;
  API_BEGIN
  if (!mesh || !mesh->coords || !mesh->tets || !partition || !eps) throw DDError{DD_ERR_ARG, "null input pointer"};
  const int64_t n_vertices = mesh->n_vertices, n_tets = mesh->n_tets;
  const double* coords = mesh->coords;
  const int32_t* tets = mesh->tets;
  if (!std::isfinite(dt) || !std::isfinite(beta)) throw DDError{DD_ERR_NONFINITE, "non-finite dt or beta"};
  if (!(dt > 0) || !(beta > 0)) throw DDError{DD_ERR_ARG, "dt and beta must be positive"};
  dd_options o;
  dd_default_options(&o);
  if (opt) o = *opt;
  if (o.nrhs < 1 || o.nrhs > kMaxRhs) throw DDError{DD_ERR_ARG, "nrhs must be in 1..32"};
  if (o.precond != 0 && o.precond != 1) throw DDError{DD_ERR_ARG, "precond must be 0 or 1"};
  if (o.method != 0 && o.method != 1) throw DDError{DD_ERR_ARG, "method must be 0 or 1"};
  if (!std::isfinite(o.robin_alpha) || o.robin_alpha < 0) throw DDError{DD_ERR_ARG, "robin_alpha must be >= 0"};
  if (o.precision != DD_FP64 && o.precision != DD_FP32_REFINE) throw DDError{DD_ERR_ARG, "unknown precision"};
  if (!(o.cg_tol > 0) || o.cg_max_iter < 1 || o.check_every < 1 || o.refine_max < 0 || !(o.refine_tol > 0))
    throw DDError{DD_ERR_ARG, "bad solver option"};
  if (o.diagnostics & ~(DD_DIAG_GAUSS | DD_DIAG_ENERGY)) throw DDError{DD_ERR_ARG, "unknown diagnostics bit"};
  for (int64_t t = 0; t < n_tets; ++t) {
    if (!std::isfinite(eps[t]) || (mu && !std::isfinite(mu[t])))
      throw DDError{DD_ERR_NONFINITE, "non-finite eps or mu at tetrahedron " + std::to_string(t)};
    if (!finite_pos(eps[t]) || (mu && !finite_pos(mu[t])))
      throw DDError{DD_ERR_ARG, "eps and mu must be positive (tetrahedron " + std::to_string(t) + ")"};
  }
  C = new Ctx();
  C->opt = o;
  C->st = (hipStream_t)o.stream;
  if (o.tune_cache) C->tune_cache = o.tune_cache;
  C->opt.tune_cache = nullptr;  // the caller's string is not kept
  HIPCHK(hipGetDevice(&C->device));
  resolve_scratch(C->device);
  HIPCHK(hipStreamCreateWithFlags(&C->st2, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&C->fa, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&C->fb, hipStreamNonBlocking));
  for (hipEvent_t* e : {&C->ev_fa, &C->ev_fb, &C->ev_ffork, &C->ev_fjoin})
    HIPCHK(hipEventCreateWithFlags(e, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&C->ev_fork, hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&C->ev_join, hipEventDisableTiming));
  C->dt = dt;
  C->beta = beta;
  C->nrhs = o.nrhs;
  C->fp32 = o.precision == DD_FP32_REFINE;
  std::string msg;
  int rc = build_plan(n_vertices, coords, n_tets, tets, partition, C->P, msg);
  if (rc != DD_OK) throw DDError{rc, msg};
  build_device(*C, coords);
  if (o.method == 1) build_dp2(*C, coords, eps, mu);
  std::vector<double> mh(n_tets, 1.0);
  if (mu) mh.assign(mu, mu + n_tets);
  HIPCHK(hipMemcpyAsync(C->d_mu, mh.data(), n_tets * sizeof(double), hipMemcpyHostToDevice, C->st));
  HIPCHK(hipMemcpyAsync(C->d_eps, eps, n_tets * sizeof(double), hipMemcpyHostToDevice, C->st));
  HIPCHK(hipStreamSynchronize(C->st));
  *out = C;
  return DD_OK;
  }
  catch (const DDError& e) {
    g_err = e.msg;
    delete C;
    return e.code;
  }
  catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    delete C;
    return DD_ERR_OOM;
  }
  catch (const std::exception& e) {
    g_err = e.what();
    delete C;
    return DD_ERR_ARG;
  }
}

int dd_get_info(void* ctx, dd_info* info) {
  if (!ctx || !info) {
    g_err = "null argument";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  std::memset(info, 0, sizeof(*info));
  info->n_edges = C.P.ne;
  info->n_interior = C.P.nint;
  info->n_tets = C.P.nt;
  info->n_vertices = C.P.nv;
  info->n_sub = C.nsub;
  info->n_lambda = (int32_t)C.nlam;
  info->n_corner = (int32_t)C.P.ncorner();
  info->nrhs = C.nrhs;
  info->precision = C.fp32 ? DD_FP32_REFINE : DD_FP64;
  info->tile = NB;
  info->factor_bytes = C.factor_bytes;
  info->trailing_bytes = C.trailing_bytes;
  info->schur_bytes = C.schur_bytes;
  info->corner_bytes = C.corner_bytes;
  info->coarse_bytes = C.coarse_bytes;
  info->full_bytes = C.full_bytes;
  info->cross_bytes = C.cross_bytes;
  return DD_OK;
}

int dd_num_edges(void* ctx, int64_t* n_edges) {
  if (!ctx || !n_edges) {
    g_err = "null argument";
    return DD_ERR_ARG;
  }
  *n_edges = ((Ctx*)ctx)->P.ne;
  return DD_OK;
}

int dd_get_edges(void* ctx, int32_t* edges, uint8_t* is_pec) {
  if (!ctx) {
    g_err = "null context";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  if (edges) std::memcpy(edges, C.P.edges.data(), C.P.edges.size() * sizeof(int32_t));
  if (is_pec) std::memcpy(is_pec, C.P.pec.data(), C.P.pec.size());
  return DD_OK;
}

int dd_set_eps(void* ctx, const double* eps_in, int on_device) {
  if (!ctx || !eps_in) {
    g_err = "null argument";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  API_BEGIN
  std::vector<double> staged;
  const double* eps = eps_in;
  if (on_device) {
    staged.resize(C.P.nt);
    HIPCHK(hipMemcpyAsync(staged.data(), eps_in, C.P.nt * sizeof(double), hipMemcpyDeviceToHost, C.st));
    HIPCHK(hipStreamSynchronize(C.st));
    eps = staged.data();
  }
  for (int64_t t = 0; t < C.P.nt; ++t) {
    if (!std::isfinite(eps[t])) throw DDError{DD_ERR_NONFINITE, "non-finite eps"};
    if (!(eps[t] > 0)) throw DDError{DD_ERR_ARG, "eps must be positive"};
  }
  HIPCHK(hipMemcpyAsync(C.d_eps, eps, C.P.nt * sizeof(double), hipMemcpyHostToDevice, C.st));
  HIPCHK(hipStreamSynchronize(C.st));
  C.factored = false;
  return DD_OK;
  API_END
}

int dd_autotune(void* ctx, const char* cache_path, dd_tuning* out) {
  if (!ctx) {
    g_err = "null context";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  if (!C.factored) {
    g_err = "dd_autotune called before dd_factor";
    return DD_ERR_STATE;
  }
  API_BEGIN
  if (C.fp32)
    autotune<float>(C, cache_path, out);
  else
    autotune<double>(C, cache_path, out);
  return DD_OK;
  API_END
}

int dd_factor(void* ctx) {
  if (!ctx) {
    g_err = "null context";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  API_BEGIN
  return C.fp32 ? factor_impl<float>(C) : factor_impl<double>(C);
  API_END
}

int dd_step(void* ctx, const double* J_half, const double* J_prev_half, const double* E_n, const double* E_nm1,
            double* E_next, dd_stats* stats) {
  if (!ctx || !J_half || !J_prev_half || !E_n || !E_nm1 || !E_next) {
    g_err = "null argument";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  if (!C.factored) {
    g_err = "dd_step called before dd_factor";
    return DD_ERR_STATE;
  }
  API_BEGIN
  int rc = C.fp32 ? step_impl<float>(C, J_half, J_prev_half, E_n, E_nm1, E_next, stats)
                  : step_impl<double>(C, J_half, J_prev_half, E_n, E_nm1, E_next, stats);
  prof_resolve(C);
  if (rc == DD_ERR_NO_CONVERGENCE) g_err = "interface CG or refinement did not reach its tolerance";
  return rc;
  API_END
}

int dd_state_set(void* ctx, const double* E_n, const double* E_nm1, const double* J_prev_half) {
  if (!ctx) {
    g_err = "null argument";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  if (!C.factored) {
    g_err = "dd_state_set called before dd_factor";
    return DD_ERR_STATE;
  }
  API_BEGIN
  resident_set(C, E_n, E_nm1, J_prev_half);
  return DD_OK;
  API_END
}

int dd_step_resident(void* ctx, const double* J_half, double* E_next, dd_stats* stats) {
  if (!ctx || !J_half || !E_next) {
    g_err = "null argument";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  if (!C.factored) {
    g_err = "dd_step_resident called before dd_factor";
    return DD_ERR_STATE;
  }
  API_BEGIN
  int rc = C.fp32 ? step_resident_impl<float>(C, J_half, E_next, stats)
                  : step_resident_impl<double>(C, J_half, E_next, stats);
  prof_resolve(C);
  if (rc == DD_ERR_NO_CONVERGENCE) g_err = "interface CG or refinement did not reach its tolerance";
  return rc;
  API_END
}

int dd_solve(void* ctx, const double* b, double* x, dd_stats* stats) {
  if (!ctx || !b || !x) {
    g_err = "null argument";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  if (!C.factored) {
    g_err = "dd_solve called before dd_factor";
    return DD_ERR_STATE;
  }
  API_BEGIN
  int rc = C.fp32 ? solve_api_impl<float>(C, b, x, stats) : solve_api_impl<double>(C, b, x, stats);
  if (rc == DD_ERR_NO_CONVERGENCE) g_err = "interface CG or refinement did not reach its tolerance";
  return rc;
  API_END
}

int dd_adjoint_step(void* ctx, const double* ebar_next, double* ebar_n, double* ebar_nm1, double* g_out,
                    const double* E_next, const double* E_n, const double* E_nm1, double* eps_bar,
                    double* Jbar_half, double* Jbar_prev_half, dd_stats* stats) {
  if (!ctx || !ebar_next || (eps_bar && (!E_next || !E_n))) {
    g_err = "null argument";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  if (!C.factored) {
    g_err = "dd_adjoint_step called before dd_factor";
    return DD_ERR_STATE;
  }
  API_BEGIN
  int rc = C.fp32 ? adjoint_impl<float>(C, ebar_next, ebar_n, ebar_nm1, g_out, E_next, E_n, E_nm1, eps_bar,
                                        Jbar_half, Jbar_prev_half, stats)
                  : adjoint_impl<double>(C, ebar_next, ebar_n, ebar_nm1, g_out, E_next, E_n, E_nm1, eps_bar,
                                         Jbar_half, Jbar_prev_half, stats);
  if (rc == DD_ERR_NO_CONVERGENCE) g_err = "interface CG or refinement did not reach its tolerance";
  return rc;
  API_END
}

int dd_set_charge(void* ctx, const double* q) {
  if (!ctx) {
    g_err = "null context";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  API_BEGIN
  const int64_t n = C.P.nv * C.nrhs;
  hipLaunchKernelGGL(k_charge_set, dim3(nblk(n)), dim3(256), 0, C.st, (int64_t)C.P.nv, C.nrhs, q, C.d_q);
  HIPCHK(hipGetLastError());
  return DD_OK;
  API_END
}

int dd_charge_update(void* ctx, const double* J_half, double* q) {
  if (!ctx || !J_half || !q) {
    g_err = "null argument";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  API_BEGIN
  int64_t n = C.P.nv * C.nrhs;
  hipLaunchKernelGGL(k_charge, dim3(nblk(n)), dim3(256), 0, C.st, (int64_t)C.P.nv, C.d_vptr, C.d_vedge,
                     C.d_nodeint, J_half, (int64_t)C.P.ne, C.dt, q, C.nrhs);
  HIPCHK(hipGetLastError());
  return DD_OK;
  API_END
}

int dd_gauss_residual(void* ctx, const double* E, const double* q, double* res) {
  if (!ctx || !E || !q || !res) {
    g_err = "null argument";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  API_BEGIN
  const int nr = C.nrhs;
  const int64_t ni = C.P.nint, ne = C.P.ne, nv = C.P.nv;
  hipLaunchKernelGGL(k_edges_to_int, dim3(nblk(ni, 64)), dim3(256), 0, C.st, ni, C.d_interior, E, ne, C.g_t1, nr,
                     1.0);
  csr_launch(C, C.st, 3, C.g_t1, nullptr, nullptr, nullptr, nullptr, 0.0, 0.0, C.g_t2, C.g_t3);
  double* d_res = C.d_vres;
  hipLaunchKernelGGL(k_gauss, dim3(nblk(nv * nr)), dim3(256), 0, C.st, nv, C.d_vptr, C.d_vedge, C.d_nodeint,
                     C.d_dof, (const double*)C.g_t2, q, nr, d_res);
  std::vector<double> h(nv * nr);
  HIPCHK(hipMemcpyAsync(h.data(), d_res, nv * nr * sizeof(double), hipMemcpyDeviceToHost, C.st));
  HIPCHK(hipStreamSynchronize(C.st));
  for (int r = 0; r < nr; ++r) {
    double m = 0.0;
    for (int64_t v = 0; v < nv; ++v) m = std::max(m, std::fabs(h[r * nv + v]));
    res[r] = m;
  }
  return DD_OK;
  API_END
}

int dd_energy(void* ctx, const double* E_next, const double* E_n, double* out) {
  if (!ctx || !E_next || !E_n || !out) {
    g_err = "null argument";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  API_BEGIN
  const int nr = C.nrhs;
  const int64_t ni = C.P.nint, ne = C.P.ne;
  hipLaunchKernelGGL(k_edges_to_int, dim3(nblk(ni, 64)), dim3(256), 0, C.st, ni, C.d_interior, E_next, ne, C.g_t1,
                     nr, 1.0);
  hipLaunchKernelGGL(k_edges_to_int, dim3(nblk(ni, 64)), dim3(256), 0, C.st, ni, C.d_interior, E_n, ne, C.g_t2, nr,
                     1.0);
  energy_int(C, C.g_t1, C.g_t2, out);
  return DD_OK;
  API_END
}

int dd_profile(void* ctx, int enable, double* ms, int64_t* launches) {
  if (!ctx) {
    g_err = "null context";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  API_BEGIN
  prof_resolve(C);
  for (int i = 0; i < DD_PROF_CLASSES; ++i) {
    if (ms) ms[i] = C.prof_ms[i];
    if (launches) launches[i] = C.prof_n[i];
  }
  if (enable >= 0) {
    C.prof = enable != 0;
    for (int i = 0; i < DD_PROF_CLASSES; ++i) {
      C.prof_ms[i] = 0.0;
      C.prof_n[i] = 0;
    }
  }
  return DD_OK;
  API_END
}

// ---- particle steps (Sec. II-A) --------------------------------------------------


int dd_pic_status(void* ctx, int64_t* counts, int reset) {
  if (!ctx) {
    g_err = "null context";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  API_BEGIN
  pic_prepare(C);
  unsigned long long c[kPicCounters];
  HIPCHK(hipMemcpyAsync(c, C.d_pic_cnt, sizeof(c), hipMemcpyDeviceToHost, C.st));
  HIPCHK(hipStreamSynchronize(C.st));
  if (counts)
    for (int k = 0; k < kPicCounters; ++k) counts[k] = (int64_t)c[k];
  if (reset) HIPCHK(hipMemsetAsync(C.d_pic_cnt, 0, sizeof(c), C.st));
  return DD_OK;
  API_END
}

int dd_pic_locate(void* ctx, int64_t n, const double* x, int32_t* cell) {
  if (!ctx || n < 0 || (n > 0 && (!x || !cell))) {
    g_err = "null argument or negative count";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  API_BEGIN
  pic_prepare(C);
  if (n == 0) return DD_OK;
  hipLaunchKernelGGL(k_pic_locate, dim3(nblk(n)), dim3(256), 0, C.st, n, (int64_t)C.P.nt, x, cell,
                     (const double*)C.d_pic_geo, (const int32_t*)C.d_pic_nbr, (const double*)C.d_coords,
                     (const int32_t*)C.d_tsort, kPicMaxCross, C.d_pic_cnt);
  HIPCHK(hipGetLastError());
  return DD_OK;
  API_END
}

int dd_pic_deposit(void* ctx, int64_t n, const double* xa, const double* xb, const double* q, int32_t* cell,
                   double* J) {
  if (!ctx || n < 0 || !J || (n > 0 && (!xa || !xb || !q || !cell))) {
    g_err = "null argument or negative count";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  API_BEGIN
  pic_prepare(C);
  if (n == 0) return DD_OK;
  hipLaunchKernelGGL(k_pic_deposit, dim3(nblk(n, kDepThreads)), dim3(kDepThreads), 0, C.st, n, (int64_t)C.P.nt, xa, xb, q, 1.0 / C.dt,
                     cell, (const double*)C.d_pic_geo, (const int32_t*)C.d_pic_nbr,
                     (const int32_t*)C.d_pic_tedge, J, kPicMaxCross, C.d_pic_cnt);
  HIPCHK(hipGetLastError());
  return DD_OK;
  API_END
}

int dd_mixed_faces(void* ctx, int64_t* n_faces, int32_t* faces) {
  if (!ctx) {
    g_err = "null context";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  API_BEGIN
  mixed_prepare(C);
  if (n_faces) *n_faces = C.n_faces;
  if (faces) std::memcpy(faces, C.faces_h.data(), C.faces_h.size() * sizeof(int32_t));
  return DD_OK;
  API_END
}

int dd_step_mixed(void* ctx, const double* J_half, const double* E_n, const double* B_n, double* E_next,
                  double* B_next, dd_stats* stats) {
  if (!ctx || !J_half || !E_n || !B_n || !E_next || !B_next) {
    g_err = "null argument";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  if (!C.factored) {
    g_err = "dd_step_mixed called before dd_factor";
    return DD_ERR_STATE;
  }
  if (C.beta != 0.25) {
    g_err = "the mixed step is the trapezoid rule: the context needs beta = 1/4";
    return DD_ERR_STATE;
  }
  if (B_next == B_n || E_next == E_n) {
    g_err = "outputs must not alias inputs";
    return DD_ERR_ARG;
  }
  API_BEGIN
  mixed_prepare(C);
  int rc = C.fp32 ? mixed_step_impl<float>(C, J_half, E_n, B_n, E_next, B_next, stats)
                  : mixed_step_impl<double>(C, J_half, E_n, B_n, E_next, B_next, stats);
  prof_resolve(C);
  if (rc == DD_ERR_NO_CONVERGENCE) g_err = "interface solve or refinement did not reach its tolerance";
  return rc;
  API_END
}

int dd_pic_sort(void* ctx, int64_t n, const int32_t* cell, int32_t* perm) {
  if (!ctx || n < 0 || (n > 0 && (!cell || !perm)) || n > INT32_MAX) {
    g_err = "null argument or count out of range";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  API_BEGIN
  pic_prepare(C);
  if (n == 0) return DD_OK;
  const int64_t nt = C.P.nt, m = nt + 1, nb = (m + kScanBlock - 1) / kScanBlock;
  // a fill kernel, not a memset: this call may be captured into a graph
  hipLaunchKernelGGL(k_zero_i32, dim3(nblk(m)), dim3(256), 0, C.st, m, C.d_pic_count);
  hipLaunchKernelGGL(k_cell_hist, dim3(nblk(n)), dim3(256), 0, C.st, n, nt, cell, C.d_pic_count);
  hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(256), 0, C.st, m, C.d_pic_count, C.d_pic_bsum);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, C.st, nb, C.d_pic_bsum);
  hipLaunchKernelGGL(k_scan_add, dim3(nblk(m)), dim3(256), 0, C.st, m, C.d_pic_count,
                     (const int32_t*)C.d_pic_bsum);
  hipLaunchKernelGGL(k_cell_scatter, dim3(nblk(n)), dim3(256), 0, C.st, n, nt, cell, C.d_pic_count, perm);
  HIPCHK(hipGetLastError());
  return DD_OK;
  API_END
}

int dd_pic_sort_noalloc(void* ctx, int64_t n, const int32_t* cell, int32_t* perm) {
  if (!ctx || n < 0 || (n > 0 && (!cell || !perm)) || n > INT32_MAX) {
    g_err = "null argument or count out of range";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  API_BEGIN
  const int64_t nt = C.P.nt, m = nt + 1, nb = (m + kScanBlock - 1) / kScanBlock;
  if (nt > kNoAllocMaxCells)
    throw DDError{DD_ERR_ARG, "the mesh has " + std::to_string(nt) + " tetrahedra; the static scratch of "
                                  "this call holds at most " + std::to_string(kNoAllocMaxCells)};
  int32_t* sc = scratch_of(C.device);
  if (!sc) throw DDError{DD_ERR_STATE, "static scratch not resolved for the context's device"};
  if (n == 0) return DD_OK;
  int32_t* count = sc;
  int32_t* bsum = sc + (kNoAllocMaxCells + 1);
  // the previous call's counts are still there: clear them with a fill
  // kernel (no memset, so the call can be captured into a graph)
  hipLaunchKernelGGL(k_zero_i32, dim3(nblk(m)), dim3(256), 0, C.st, m, count);
  hipLaunchKernelGGL(k_cell_hist, dim3(nblk(n)), dim3(256), 0, C.st, n, nt, cell, count);
  hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(256), 0, C.st, m, count, bsum);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, C.st, nb, bsum);
  hipLaunchKernelGGL(k_scan_add, dim3(nblk(m)), dim3(256), 0, C.st, m, count, (const int32_t*)bsum);
  hipLaunchKernelGGL(k_cell_scatter, dim3(nblk(n)), dim3(256), 0, C.st, n, nt, cell, count, perm);
  HIPCHK(hipGetLastError());
  return DD_OK;
  API_END
}

int dd_pic_permute(void* ctx, int64_t n, const int32_t* perm, int item_bytes, const void* src, void* dst) {
  if (!ctx || n < 0 || (n > 0 && (!perm || !src || !dst)) || item_bytes <= 0 || item_bytes > 64 ||
      item_bytes % 4 != 0) {
    g_err = "null argument, negative count or item size not a multiple of 4 in [4, 64]";
    return DD_ERR_ARG;
  }
  if (n > 0 && src == dst) {
    g_err = "src and dst must differ";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  API_BEGIN
  pic_prepare(C);
  if (n == 0) return DD_OK;
  const int words = item_bytes / 4;
  hipLaunchKernelGGL(k_permute, dim3(nblk(n * words)), dim3(256), 0, C.st, n, words, perm, (const uint32_t*)src,
                     (uint32_t*)dst, C.d_pic_cnt);
  HIPCHK(hipGetLastError());
  return DD_OK;
  API_END
}

int dd_pic_faraday(void* ctx, int nrows, const double* E, double alpha, double* B) {
  if (!ctx || !E || !B || nrows < 1) {
    g_err = "null argument or nrows < 1";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  API_BEGIN
  pic_prepare(C);
  hipLaunchKernelGGL(k_pic_faraday, dim3(nblk(C.P.nt)), dim3(256), 0, C.st, (int64_t)C.P.nt, nrows, (int64_t)C.P.ne,
                     E, alpha, (const double*)C.d_pic_geo, (const int32_t*)C.d_pic_tedge, B);
  HIPCHK(hipGetLastError());
  return DD_OK;
  API_END
}

int dd_pic_push(void* ctx, int64_t n, const double* qm, const double* E, const double* B, const int32_t* cell,
                const double* x, double* x_new, double* v, double* hist, int first) {
  if (!ctx || n < 0 || (n > 0 && (!qm || !E || !B || !cell || !x || !x_new || !v || !hist))) {
    g_err = "null argument or negative count";
    return DD_ERR_ARG;
  }
  if (n > 0 && x_new == x) {
    g_err = "x_new must not be x";
    return DD_ERR_ARG;
  }
  Ctx& C = *(Ctx*)ctx;
  API_BEGIN
  pic_prepare(C);
  if (n > 0)
    hipLaunchKernelGGL(k_pic_push, dim3(nblk(n)), dim3(256), 0, C.st, n, (int64_t)C.P.nt, qm, E, B, cell, x, x_new,
                       v, hist, (const double*)C.d_pic_geo, (const int32_t*)C.d_pic_tedge, C.dt, first ? 1 : 0,
                       C.d_pic_cnt);
  HIPCHK(hipGetLastError());
  return DD_OK;
  API_END
}

void dd_destroy(void* ctx) { delete (Ctx*)ctx; }

int dd_analyze(const dd_mesh* mesh, const int32_t* partition, dd_analysis* out, int32_t* per_sub) {
  g_err.clear();
  if (!out || !mesh) {
    g_err = "out or mesh is NULL";
    return DD_ERR_ARG;
  }
  API_BEGIN
  Plan P;
  std::string msg;
  int rc = build_plan(mesh->n_vertices, mesh->coords, mesh->n_tets, mesh->tets, partition, P, msg);
  if (rc != DD_OK) throw DDError{rc, msg};
  std::memset(out, 0, sizeof(*out));
  out->n_edges = P.ne;
  out->n_interior = P.nint;
  out->n_sub = P.nsub;
  out->n_lambda = (int32_t)P.nlambda();
  out->n_corner = (int32_t)P.ncorner();
  out->max_multiplicity = P.max_mult;
  for (int s = 0; s < P.nsub; ++s) {
    int64_t nr = P.subs[s].nI + P.subs[s].nG;
    out->sum_nr3 += nr * nr * nr;
    if (per_sub) {
      per_sub[3 * s] = P.subs[s].nI;
      per_sub[3 * s + 1] = P.subs[s].nG;
      per_sub[3 * s + 2] = P.subs[s].nC;
    }
  }
  return DD_OK;
  API_END
}

int dd_analyze_lambda(const dd_mesh* mesh, const int32_t* partition, int32_t* edge, int32_t* sub_lo,
                      int32_t* sub_hi, int32_t* pos_lo, int32_t* pos_hi) {
  g_err.clear();
  if (!mesh) {
    g_err = "mesh is NULL";
    return DD_ERR_ARG;
  }
  API_BEGIN
  Plan P;
  std::string msg;
  int rc = build_plan(mesh->n_vertices, mesh->coords, mesh->n_tets, mesh->tets, partition, P, msg);
  if (rc != DD_OK) throw DDError{rc, msg};
  for (int64_t l = 0; l < P.nlambda(); ++l) {
    if (edge) edge[l] = P.interior[P.lam_dof[l]];
    if (sub_lo) sub_lo[l] = P.lam_s0[l];
    if (sub_hi) sub_hi[l] = P.lam_s1[l];
    if (pos_lo) pos_lo[l] = P.lam_p0[l];
    if (pos_hi) pos_hi[l] = P.lam_p1[l];
  }
  return DD_OK;
  API_END
}

}  // extern "C"

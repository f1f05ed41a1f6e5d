// Host-side partition analysis; see plan.hpp.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

#include "ddfem.h"

namespace ddfem {

namespace {
const int LE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

template <class T>
void sort_unique(std::vector<T>& v) {
  std::sort(v.begin(), v.end());
  v.erase(std::unique(v.begin(), v.end()), v.end());
}
}  // namespace

// Nested dissection of a point set carrying a graph (items 0..n-1 with
// coordinates mid[3i..3i+2] and adjacency adj[i]): split at the median
// coordinate of the widest axis; items of the lower side with a neighbour on
// the upper side form the separator, ordered after both halves.  Pieces of
// at most `leaf` items keep their incoming order.  Returns order[k] = item
// placed at position k.
static std::vector<int32_t> dissect(int32_t n, const std::vector<double>& mid,
                                    const std::vector<std::vector<int32_t>>& adj, size_t leaf) {
  std::vector<int32_t> order;
  order.reserve(n);
  std::vector<uint8_t> side(n, 0);
  // explicit recursion; a frame orders (left interior, right, separator)
  struct Frame {
    std::vector<int32_t> idx;
    int stage;
    std::vector<int32_t> right, sep;
  };
  std::vector<Frame> st;
  std::vector<int32_t> all(n);
  std::iota(all.begin(), all.end(), 0);
  st.push_back({all, 0, {}, {}});
  while (!st.empty()) {
    Frame& f = st.back();
    if (f.stage == 0) {
      if (f.idx.size() <= leaf) {
        order.insert(order.end(), f.idx.begin(), f.idx.end());
        st.pop_back();
        continue;
      }
      double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
      for (int32_t c : f.idx)
        for (int k = 0; k < 3; ++k) {
          lo[k] = std::min(lo[k], mid[3 * c + k]);
          hi[k] = std::max(hi[k], mid[3 * c + k]);
        }
      int ax = 0;
      for (int k = 1; k < 3; ++k)
        if (hi[k] - lo[k] > hi[ax] - lo[ax]) ax = k;
      std::vector<double> xs;
      xs.reserve(f.idx.size());
      for (int32_t c : f.idx) xs.push_back(mid[3 * c + ax]);
      std::nth_element(xs.begin(), xs.begin() + xs.size() / 2, xs.end());
      const double med = xs[xs.size() / 2];
      std::vector<int32_t> left, right;
      for (int32_t c : f.idx) (mid[3 * c + ax] < med ? left : right).push_back(c);
      if (left.empty() || right.empty()) {
        order.insert(order.end(), f.idx.begin(), f.idx.end());
        st.pop_back();
        continue;
      }
      for (int32_t c : right) side[c] = 2;
      std::vector<int32_t> lint, sep;
      for (int32_t c : left) {
        bool cut = false;
        for (int32_t d : adj[c])
          if (side[d] == 2) {
            cut = true;
            break;
          }
        (cut ? sep : lint).push_back(c);
      }
      for (int32_t c : right) side[c] = 0;
      f.stage = 1;
      f.right = std::move(right);
      f.sep = std::move(sep);
      std::vector<int32_t> l2 = std::move(lint);
      st.push_back({std::move(l2), 0, {}, {}});
    } else if (f.stage == 1) {
      f.stage = 2;
      std::vector<int32_t> r = std::move(f.right);
      st.push_back({std::move(r), 0, {}, {}});
    } else {
      order.insert(order.end(), f.sep.begin(), f.sep.end());
      st.pop_back();
    }
  }
  return order;
}

static void edge_midpoint(const Plan& P, const double* coords, int32_t d, double* m) {
  int32_t e = P.interior[d];
  for (int k = 0; k < 3; ++k)
    m[k] = 0.5 * (coords[3 * (int64_t)P.edges[2 * e] + k] + coords[3 * (int64_t)P.edges[2 * e + 1] + k]);
}

// Fill-reducing order of the corner unknowns (the coarse problem).  The
// coarse matrix K_cc = sum_s B_c^T K_s B_c couples every pair of corners of
// one subdomain; nested dissection of that graph by coordinate bisection of
// the corner-edge midpoints.  Only the fill of the coarse factor and of its
// inverse depends on this order (the solve stores and streams only nonzero
// tiles).
static void order_corners(Plan& P, const double* coords) {
  const int64_t nc = P.ncorner();
  if (nc == 0) return;
  std::vector<std::vector<int32_t>> adj(nc);
  for (int32_t s = 0; s < P.nsub; ++s) {
    const SubInfo& q = P.subs[s];
    const auto& L = P.local[s];
    for (int32_t a = 0; a < q.nC; ++a) {
      int32_t I = P.dof_corner[L[q.nI + q.nG + a]];
      for (int32_t b = 0; b < q.nC; ++b)
        if (a != b) adj[I].push_back(P.dof_corner[L[q.nI + q.nG + b]]);
    }
  }
  for (auto& v : adj) sort_unique(v);
  std::vector<double> mid(3 * nc);
  for (int64_t c = 0; c < nc; ++c) edge_midpoint(P, coords, P.corner_dof[c], &mid[3 * c]);
  std::vector<int32_t> order = dissect((int32_t)nc, mid, adj, 64);
  std::vector<int32_t> cd(nc);
  for (int64_t k = 0; k < nc; ++k) cd[k] = P.corner_dof[order[k]];
  P.corner_dof = cd;
  for (int64_t k = 0; k < nc; ++k) P.dof_corner[cd[k]] = (int32_t)k;
}

// Order of each subdomain's interior block.  The interior unknowns are
// eliminated first (Sec. III-C); their order changes only the fill of
// L_rr and of the stored inverse L_rr^-1.  Nested dissection of the local
// coupling graph (two interior unknowns couple when they share a tet of the
// subdomain) makes whole tiles of L_II^-1 zero: the inverse factor couples
// an unknown only to its ancestors in the dissection tree, so the two halves
// of every dissection stay uncoupled.
static void order_interiors(Plan& P, const double* coords, const int32_t* partition) {
  std::vector<int64_t> tptr(P.nsub + 1, 0), tlist(P.nt);
  for (int64_t t = 0; t < P.nt; ++t) tptr[partition[t] + 1]++;
  for (int32_t s = 0; s < P.nsub; ++s) tptr[s + 1] += tptr[s];
  {
    std::vector<int64_t> fill(tptr.begin(), tptr.end() - 1);
    for (int64_t t = 0; t < P.nt; ++t) tlist[fill[partition[t]]++] = t;
  }
  std::vector<int32_t> loc(P.nint, -1);
  for (int32_t s = 0; s < P.nsub; ++s) {
    const int32_t nI = P.subs[s].nI;
    if (nI <= 64) continue;
    auto& L = P.local[s];
    for (int32_t a = 0; a < nI; ++a) loc[L[a]] = a;
    std::vector<std::vector<int32_t>> adj(nI);
    for (int64_t k = tptr[s]; k < tptr[s + 1]; ++k) {
      const int64_t t = tlist[k];
      int32_t li[6];
      for (int e = 0; e < 6; ++e) {
        int32_t d = P.dof[P.tet_edges[t * 6 + e]];
        li[e] = d >= 0 ? loc[d] : -1;
      }
      for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b)
          if (a != b && li[a] >= 0 && li[b] >= 0) adj[li[a]].push_back(li[b]);
    }
    for (auto& v : adj) sort_unique(v);
    std::vector<double> mid(3 * (size_t)nI);
    for (int32_t a = 0; a < nI; ++a) edge_midpoint(P, coords, L[a], &mid[3 * a]);
    std::vector<int32_t> order = dissect(nI, mid, adj, 64);
    std::vector<int32_t> seg(nI);
    for (int32_t k = 0; k < nI; ++k) seg[k] = L[order[k]];
    for (int32_t a = 0; a < nI; ++a) loc[L[a]] = -1;
    std::copy(seg.begin(), seg.end(), L.begin());
  }
}

// Order of each subdomain's interface and corner blocks.  It changes only
// how the couplings L_GI and L_cI of the factor fall into tiles: the
// nonzero pattern of a row of L_GI is a property of that row alone (the
// dissection pieces of the interior that the unknown shares a tet with, and
// the separators above them).  Rows are sorted by the first interior
// position (in the dissection order) that they touch, so the rows next to
// one piece sit together and share its tiles instead of spreading a few
// nonzero rows over many tiles.  Ties keep ascending unknown id; rows that
// touch no interior unknown go last.  The multipliers' local positions are
// moved with their rows.
static void order_boundary(Plan& P, const int32_t* partition) {
  std::vector<int64_t> tptr(P.nsub + 1, 0), tlist(P.nt);
  for (int64_t t = 0; t < P.nt; ++t) tptr[partition[t] + 1]++;
  for (int32_t s = 0; s < P.nsub; ++s) tptr[s + 1] += tptr[s];
  {
    std::vector<int64_t> fill(tptr.begin(), tptr.end() - 1);
    for (int64_t t = 0; t < P.nt; ++t) tlist[fill[partition[t]]++] = t;
  }
  std::vector<int32_t> ipos(P.nint, -1), key(P.nint, INT32_MAX);
  // moved[s][old position - nI] = new position of the interface / corner row
  std::vector<std::vector<int32_t>> moved(P.nsub);
  for (int32_t s = 0; s < P.nsub; ++s) {
    const SubInfo& q = P.subs[s];
    auto& L = P.local[s];
    for (int32_t a = 0; a < q.nI; ++a) ipos[L[a]] = a;
    for (int64_t k = tptr[s]; k < tptr[s + 1]; ++k) {
      const int64_t t = tlist[k];
      int32_t d[6];
      for (int e = 0; e < 6; ++e) d[e] = P.dof[P.tet_edges[t * 6 + e]];
      for (int a = 0; a < 6; ++a) {
        if (d[a] < 0 || ipos[d[a]] < 0) continue;
        for (int b = 0; b < 6; ++b)
          if (d[b] >= 0 && ipos[d[b]] < 0) key[d[b]] = std::min(key[d[b]], ipos[d[a]]);
      }
    }
    auto& mv = moved[s];
    mv.resize(q.nG + q.nC);
    for (int seg = 0; seg < 2; ++seg) {
      const int32_t b = seg == 0 ? q.nI : q.nI + q.nG, n = seg == 0 ? q.nG : q.nC;
      std::vector<int32_t> idx(n);
      std::iota(idx.begin(), idx.end(), 0);
      // the segment is ascending by unknown id: a stable sort keeps that
      // order among equal keys
      std::stable_sort(idx.begin(), idx.end(),
                       [&](int32_t x, int32_t y) { return key[L[b + x]] < key[L[b + y]]; });
      std::vector<int32_t> seg_new(n);
      for (int32_t k = 0; k < n; ++k) {
        seg_new[k] = L[b + idx[k]];
        mv[b + idx[k] - q.nI] = b + k;
      }
      std::copy(seg_new.begin(), seg_new.end(), L.begin() + b);
    }
    for (int32_t a = 0; a < q.nI; ++a) ipos[L[a]] = -1;
    for (int32_t a = q.nI; a < q.nI + q.nG + q.nC; ++a) key[L[a]] = INT32_MAX;
  }
  for (size_t l = 0; l < P.lam_dof.size(); ++l) {
    P.lam_p0[l] = moved[P.lam_s0[l]][P.lam_p0[l] - P.subs[P.lam_s0[l]].nI];
    P.lam_p1[l] = moved[P.lam_s1[l]][P.lam_p1[l] - P.subs[P.lam_s1[l]].nI];
  }
}

int build_plan(int64_t nv, const double* coords, int64_t nt, const int32_t* tets,
               const int32_t* partition, Plan& P, std::string& msg) {
  if (nv <= 0 || nt <= 0 || !coords || !tets || !partition) {
    msg = "empty mesh or null pointer";
    return DD_ERR_ARG;
  }
  if (nv >= (int64_t(1) << 21) * 64) {
    msg = "too many vertices";
    return DD_ERR_ARG;
  }
  P.nv = nv;
  P.nt = nt;
  P.tsort.resize(nt * 4);
  // ---- tetrahedra: range, distinct vertices, volume --------------------
  for (int64_t t = 0; t < nt; ++t) {
    int32_t v[4];
    for (int a = 0; a < 4; ++a) {
      v[a] = tets[t * 4 + a];
      if (v[a] < 0 || v[a] >= nv) {
        msg = "tetrahedron " + std::to_string(t) + " has a vertex index out of range";
        return DD_ERR_MESH;
      }
    }
    std::sort(v, v + 4);
    for (int a = 0; a < 3; ++a)
      if (v[a] == v[a + 1]) {
        msg = "tetrahedron " + std::to_string(t) + " repeats a vertex";
        return DD_ERR_MESH;
      }
    double d[3][3], scale = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) {
        double x = coords[3 * (int64_t)v[a + 1] + c], x0 = coords[3 * (int64_t)v[0] + c];
        if (!std::isfinite(x) || !std::isfinite(x0)) {
          msg = "non-finite vertex coordinate";
          return DD_ERR_NONFINITE;
        }
        d[a][c] = x - x0;
        scale = std::max(scale, std::fabs(d[a][c]));
      }
    double det = d[0][0] * (d[1][1] * d[2][2] - d[1][2] * d[2][1]) -
                 d[0][1] * (d[1][0] * d[2][2] - d[1][2] * d[2][0]) +
                 d[0][2] * (d[1][0] * d[2][1] - d[1][1] * d[2][0]);
    if (!(std::fabs(det) > 1e-12 * scale * scale * scale)) {
      msg = "tetrahedron " + std::to_string(t) + " is degenerate (zero volume)";
      return DD_ERR_MESH;
    }
    for (int a = 0; a < 4; ++a) P.tsort[t * 4 + a] = v[a];
  }
  // ---- partition ----------------------------------------------------------
  int32_t nsub = 0;
  for (int64_t t = 0; t < nt; ++t) {
    if (partition[t] < 0) {
      msg = "negative subdomain id";
      return DD_ERR_PARTITION;
    }
    nsub = std::max(nsub, partition[t] + 1);
  }
  if (nsub > (1 << 20)) {
    msg = "subdomain id out of range";
    return DD_ERR_PARTITION;
  }
  {
    std::vector<int64_t> cnt(nsub, 0);
    for (int64_t t = 0; t < nt; ++t) cnt[partition[t]]++;
    for (int32_t s = 0; s < nsub; ++s)
      if (cnt[s] == 0) {
        msg = "subdomain " + std::to_string(s) + " is empty";
        return DD_ERR_PARTITION;
      }
  }
  P.nsub = nsub;
  P.part.assign(partition, partition + nt);

  // ---- canonical edges ----------------------------------------------------------
  const uint64_t NV = (uint64_t)nv;
  std::vector<uint64_t> keys(nt * 6);
  for (int64_t t = 0; t < nt; ++t)
    for (int e = 0; e < 6; ++e)
      keys[t * 6 + e] = (uint64_t)P.tsort[t * 4 + LE[e][0]] * NV + P.tsort[t * 4 + LE[e][1]];
  std::vector<uint64_t> ukeys = keys;
  sort_unique(ukeys);
  P.ne = (int64_t)ukeys.size();
  P.edges.resize(P.ne * 2);
  for (int64_t e = 0; e < P.ne; ++e) {
    P.edges[2 * e] = (int32_t)(ukeys[e] / NV);
    P.edges[2 * e + 1] = (int32_t)(ukeys[e] % NV);
  }
  P.tet_edges.resize(nt * 6);
  for (int64_t i = 0; i < nt * 6; ++i)
    P.tet_edges[i] = (int32_t)(std::lower_bound(ukeys.begin(), ukeys.end(), keys[i]) - ukeys.begin());
  keys.clear();
  keys.shrink_to_fit();

  // ---- boundary faces -> PEC edges and boundary vertices ------------------------
  {
    const int LF[4][3] = {{0, 1, 2}, {0, 1, 3}, {0, 2, 3}, {1, 2, 3}};
    std::vector<uint64_t> fk(nt * 4);
    for (int64_t t = 0; t < nt; ++t)
      for (int f = 0; f < 4; ++f)
        fk[t * 4 + f] = ((uint64_t)P.tsort[t * 4 + LF[f][0]] * NV + P.tsort[t * 4 + LF[f][1]]) * NV +
                        P.tsort[t * 4 + LF[f][2]];
    std::sort(fk.begin(), fk.end());
    P.pec.assign(P.ne, 0);
    P.node_interior.assign(nv, 1);
    for (size_t i = 0; i < fk.size();) {
      size_t j = i;
      while (j < fk.size() && fk[j] == fk[i]) ++j;
      if (j - i == 1) {  // boundary face
        uint64_t k = fk[i];
        int32_t c = (int32_t)(k % NV), b = (int32_t)((k / NV) % NV), a = (int32_t)(k / NV / NV);
        int32_t vs[3] = {a, b, c};
        for (int x = 0; x < 3; ++x) P.node_interior[vs[x]] = 0;
        const int FE[3][2] = {{0, 1}, {0, 2}, {1, 2}};
        for (int x = 0; x < 3; ++x) {
          uint64_t ek = (uint64_t)vs[FE[x][0]] * NV + vs[FE[x][1]];
          int64_t e = std::lower_bound(ukeys.begin(), ukeys.end(), ek) - ukeys.begin();
          P.pec[e] = 1;
        }
      } else if (j - i > 2) {
        msg = "a face is shared by more than two tetrahedra";
        return DD_ERR_MESH;
      }
      i = j;
    }
  }
  P.dof.assign(P.ne, -1);
  P.interior.clear();
  for (int64_t e = 0; e < P.ne; ++e)
    if (!P.pec[e]) {
      P.dof[e] = (int32_t)P.interior.size();
      P.interior.push_back((int32_t)e);
    }
  P.nint = (int64_t)P.interior.size();

  // ---- multiplicity, owner, per-subdomain unknown sets ----------------------------
  std::vector<uint64_t> sd;  // (subdomain << 32) | unknown
  sd.reserve(nt * 6);
  for (int64_t t = 0; t < nt; ++t)
    for (int e = 0; e < 6; ++e) {
      int32_t d = P.dof[P.tet_edges[t * 6 + e]];
      if (d >= 0) sd.push_back(((uint64_t)partition[t] << 32) | (uint32_t)d);
    }
  sort_unique(sd);
  P.mult.assign(P.nint, 0);
  P.owner.assign(P.nint, INT32_MAX);
  for (uint64_t k : sd) {
    int32_t s = (int32_t)(k >> 32), d = (int32_t)(k & 0xffffffffu);
    P.mult[d]++;
    P.owner[d] = std::min(P.owner[d], s);
  }
  P.max_mult = 0;
  for (int64_t d = 0; d < P.nint; ++d) P.max_mult = std::max(P.max_mult, P.mult[d]);

  P.subs.assign(nsub, SubInfo());
  P.local.assign(nsub, {});
  {
    std::vector<std::vector<int32_t>> cls[3];
    for (int c = 0; c < 3; ++c) cls[c].assign(nsub, {});
    for (uint64_t k : sd) {
      int32_t s = (int32_t)(k >> 32), d = (int32_t)(k & 0xffffffffu);
      int c = P.mult[d] == 1 ? 0 : (P.mult[d] == 2 ? 1 : 2);
      cls[c][s].push_back(d);  // ascending unknown id = ascending edge id
    }
    for (int32_t s = 0; s < nsub; ++s) {
      SubInfo& q = P.subs[s];
      q.nI = (int32_t)cls[0][s].size();
      q.nG = (int32_t)cls[1][s].size();
      q.nC = (int32_t)cls[2][s].size();
      q.kI = (q.nI + NB - 1) / NB;
      q.kG = (q.nG + NB - 1) / NB;
      q.kC = (q.nC + NB - 1) / NB;
      q.K = q.kI + q.kG + q.kC;
      auto& L = P.local[s];
      L.reserve(q.nI + q.nG + q.nC);
      for (int c = 0; c < 3; ++c) L.insert(L.end(), cls[c][s].begin(), cls[c][s].end());
    }
  }
  sd.clear();
  sd.shrink_to_fit();

  // ---- multipliers: one per interface unknown -----------------------------------
  // position lookup per (subdomain, unknown): binary search in the class
  // segments of the local list
  auto local_pos = [&](int32_t s, int32_t d) -> int32_t {
    const SubInfo& q = P.subs[s];
    const auto& L = P.local[s];
    int c = P.mult[d] == 1 ? 0 : (P.mult[d] == 2 ? 1 : 2);
    int32_t b = c == 0 ? 0 : (c == 1 ? q.nI : q.nI + q.nG);
    int32_t e = c == 0 ? q.nI : (c == 1 ? q.nI + q.nG : q.nI + q.nG + q.nC);
    auto it = std::lower_bound(L.begin() + b, L.begin() + e, d);
    return (int32_t)(it - L.begin());
  };
  {
    // subdomains of each interface unknown: scan tets again (cheap)
    std::vector<int32_t> s0(P.nint, INT32_MAX), s1(P.nint, -1);
    for (int64_t t = 0; t < nt; ++t)
      for (int e = 0; e < 6; ++e) {
        int32_t d = P.dof[P.tet_edges[t * 6 + e]];
        if (d < 0 || P.mult[d] != 2) continue;
        s0[d] = std::min(s0[d], partition[t]);
        s1[d] = std::max(s1[d], partition[t]);
      }
    P.lam_dof.clear();
    for (int64_t d = 0; d < P.nint; ++d)
      if (P.mult[d] == 2) {
        P.lam_dof.push_back((int32_t)d);
        P.lam_s0.push_back(s0[d]);
        P.lam_s1.push_back(s1[d]);
        P.lam_p0.push_back(local_pos(s0[d], (int32_t)d));
        P.lam_p1.push_back(local_pos(s1[d], (int32_t)d));
      }
  }
  P.dof_corner.assign(P.nint, -1);
  P.corner_dof.clear();
  for (int64_t d = 0; d < P.nint; ++d)
    if (P.mult[d] >= 3) {
      P.dof_corner[d] = (int32_t)P.corner_dof.size();
      P.corner_dof.push_back((int32_t)d);
    }
  order_corners(P, coords);
  order_interiors(P, coords, partition);
  order_boundary(P, partition);
  return DD_OK;
}

int face_neighbors(const Plan& P, std::vector<int32_t>& nbr, std::string& msg) {
  struct Face {
    int32_t a, b, c;  // vertices ascending
    int32_t slot;     // 4t + opposite local vertex
  };
  const int64_t nt = P.nt;
  std::vector<Face> f((size_t)nt * 4);
  for (int64_t t = 0; t < nt; ++t) {
    const int32_t* v = &P.tsort[t * 4];
    for (int k = 0; k < 4; ++k) {
      int32_t w[3], m = 0;
      for (int i = 0; i < 4; ++i)
        if (i != k) w[m++] = v[i];
      f[t * 4 + k] = Face{w[0], w[1], w[2], (int32_t)(t * 4 + k)};
    }
  }
  std::sort(f.begin(), f.end(), [](const Face& x, const Face& y) {
    if (x.a != y.a) return x.a < y.a;
    if (x.b != y.b) return x.b < y.b;
    if (x.c != y.c) return x.c < y.c;
    return x.slot < y.slot;
  });
  nbr.assign((size_t)nt * 4, -1);
  for (size_t i = 0; i < f.size();) {
    size_t j = i;
    while (j < f.size() && f[j].a == f[i].a && f[j].b == f[i].b && f[j].c == f[i].c) ++j;
    if (j - i > 2) {
      msg = "a face is shared by more than two tetrahedra";
      return DD_ERR_MESH;
    }
    if (j - i == 2) {
      nbr[f[i].slot] = f[i + 1].slot / 4;
      nbr[f[i + 1].slot] = f[i].slot / 4;
    }
    i = j;
  }
  return 0;
}

}  // namespace ddfem

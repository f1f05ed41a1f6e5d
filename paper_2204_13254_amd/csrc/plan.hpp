// Host-side partition analysis (integer work, once per context).
//
// Sec. III: the mesh is torn into non-overlapping subdomains; unknowns are
// split into those private to one subdomain (interior, I), those shared by
// exactly two (interface, Gamma; tied by one Lagrange multiplier with a
// signed Boolean map B_r, +1 in the lower subdomain id and -1 in the higher)
// and those shared by three or more (corners, c; kept primal and gathered
// by the unsigned map B_c).  Each subdomain orders its unknowns
// [I | Gamma | c]: Gamma and c in ascending canonical edge id, I in a
// nested-dissection order of the local coupling graph (fill of the stored
// inverse factor only).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ddfem {

constexpr int NB = 32;  // tile edge of every dense block store

struct SubInfo {
  int32_t nI = 0, nG = 0, nC = 0;      // unpadded class sizes
  int32_t kI = 0, kG = 0, kC = 0, K = 0;  // tile counts per class (K = kI+kG+kC)
  int64_t tile_off = 0;                // first tile of the packed lower triangle
  int64_t row_off = 0;                 // first row of the local vector block (K*NB rows)
  int32_t kr() const { return kI + kG; }
};

struct Plan {
  int64_t nv = 0, nt = 0;
  std::vector<int32_t> tsort;       // [nt][4] vertices ascending
  std::vector<int32_t> edges;       // [ne][2] canonical edges
  std::vector<uint8_t> pec;         // [ne]
  std::vector<int32_t> tet_edges;   // [nt][6] local edges 01,02,03,12,13,23 -> edge id
  int64_t ne = 0, nint = 0;
  std::vector<int32_t> dof;         // [ne] edge -> unknown id or -1
  std::vector<int32_t> interior;    // [nint] unknown -> edge
  std::vector<uint8_t> node_interior;  // [nv] vertex not on a boundary face
  int32_t nsub = 0;
  std::vector<int32_t> part;        // [nt]
  std::vector<int32_t> mult;        // [nint] number of subdomains touching the unknown
  std::vector<int32_t> owner;       // [nint] lowest subdomain id touching it
  std::vector<SubInfo> subs;        // [nsub]
  std::vector<std::vector<int32_t>> local;   // per subdomain: unpadded local -> unknown
  // interface multipliers
  std::vector<int32_t> lam_dof, lam_s0, lam_s1, lam_p0, lam_p1;  // p: unpadded local pos
  // corners
  std::vector<int32_t> corner_dof;  // [ncorner]
  std::vector<int32_t> dof_corner;  // [nint] -> corner id or -1
  int32_t max_mult = 0;

  int64_t nlambda() const { return (int64_t)lam_dof.size(); }
  int64_t ncorner() const { return (int64_t)corner_dof.size(); }
  // padded local row of unpadded position p in subdomain s
  int32_t padded_row(int s, int32_t p) const {
    const SubInfo& q = subs[s];
    if (p < q.nI) return p;
    if (p < q.nI + q.nG) return q.kI * NB + (p - q.nI);
    return q.kr() * NB + (p - q.nI - q.nG);
  }
};

// Face neighbours of the sorted tetrahedra: nbr[4t + k] is the tetrahedron
// that shares the face opposite local vertex k of t, or -1 on the outer
// boundary.  Returns 0 or DD_ERR_MESH (a face shared by more than two).
int face_neighbors(const Plan& P, std::vector<int32_t>& nbr, std::string& msg);

// Returns 0 or a dd_status; msg receives the error text.
int build_plan(int64_t nv, const double* coords, int64_t nt, const int32_t* tets,
               const int32_t* partition, Plan& plan, std::string& msg);

}  // namespace ddfem

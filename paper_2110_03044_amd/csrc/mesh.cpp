// Host-side mesh preprocessing: validation of the face-to-cell incidence and the tables the
// kernels read.  Everything here runs once per mesh, before any time loop.
//
// From the incidence (own, nbr) and the unit face normals this builds, in mesh order:
//   * the cell -> face lists (the transpose E_{F->C} of the oriented incidence, Section 2),
//     each list in ascending face order with the orientation in the index sign;
//   * per face and side the far-upwind cell: for C = own (flow along the normal) and for
//     C = nbr (flow against it), the faces j != f of C are projected on the normal of f with
//     weight w_j = s (n_f . t_j), t_j the normal of j oriented into C.  This is the upstream
//     adjacency A^U_FF = (A_FF - Q A^D_FF)/2 of Section 3.1 applied through the normal matrices
//     (d_U = Q N (I (x) A^U) N^T E theta), precomputed once as the paper precomputes S_{C->F} and
//     T_{C->F}.  Where every side has exactly one face with weight 1 (hexahedra,
//     quadrilaterals and lines, in any numbering) d_U is theta_C - theta_U and one far cell per
//     side is kept; otherwise (triangles, tetrahedra, skewed cells) every side keeps its list of
//     (far cell, weight) pairs;
//   * where every cell's faces form opposite pairs, the per-cell slot tables of the fused kernel;
//   * optionally a renumbering for gather locality (space-filling curve or breadth-first).
//
// The loops over faces, cells and tiles run on the host's cores (OpenMP).  Every parallel loop
// writes disjoint outputs or reduces with min / max / and, and every sort has unique keys, so
// the tables (and the first error reported) are the same for any thread count.
//
// With the environment variable FL_MESH_PROGRESS set, each phase reports its wall time on
// stderr (a mesh of 10^8 cells takes minutes).
#include <omp.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <numeric>
#include <parallel/algorithm>
#include <sstream>

#include "fl_internal.h"

namespace fl {
namespace {

// Phase timing on stderr when FL_MESH_PROGRESS is set.
class Progress {
  public:
    Progress() : on_(std::getenv("FL_MESH_PROGRESS") != nullptr), t_(now()) {}
    void operator()(const char *phase, int64_t nc) {
        if (!on_) return;
        const double t = now();
        std::fprintf(stderr, "fl_mesh_create: %s (%lld cells) %.1f s\n", phase, (long long)nc,
                     t - t_);
        std::fflush(stderr);
        t_ = t;
    }

  private:
    static double now() {
        return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
            .count();
    }
    bool on_;
    double t_;
};

constexpr double kNormTol = 1e-12;

struct Csr {
    std::vector<int64_t> ptr;  // [C+1]
    std::vector<int32_t> idx;  // faces of each cell, ascending
};

// A boundary face (nbr == -1) is in its one cell's list only.
Csr cell_faces(int64_t nc, int64_t nf, const int32_t *fc) {
    Csr c;
    c.ptr.assign(nc + 1, 0);
    int64_t *ptr = c.ptr.data();
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < nf; ++f) {
#pragma omp atomic
        ptr[fc[2 * f] + 1]++;
        if (fc[2 * f + 1] >= 0) {
#pragma omp atomic
            ptr[fc[2 * f + 1] + 1]++;
        }
    }
    for (int64_t i = 0; i < nc; ++i) ptr[i + 1] += ptr[i];
    c.idx.resize(ptr[nc]);
    std::vector<int64_t> fill(c.ptr.begin(), c.ptr.end() - 1);
    int64_t *fl = fill.data();
    int32_t *idx = c.idx.data();
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < nf; ++f)
        for (int side = 0; side < 2; ++side) {
            if (fc[2 * f + side] < 0) continue;
            int64_t at;
#pragma omp atomic capture
            at = fl[fc[2 * f + side]]++;
            idx[at] = (int32_t)f;
        }
    // each list in ascending face order, whatever order the threads filled it in
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nc; ++i) std::sort(idx + ptr[i], idx + ptr[i + 1]);
    return c;
}

inline int32_t other(const int32_t *fc, int64_t f, int64_t c) {
    return fc[2 * f] == c ? fc[2 * f + 1] : fc[2 * f];
}

// FL_OK, or the status for invalid face f (reported through fail() when `report`).
fl_status check_face(int64_t nc, const int32_t *fc, const double *nrm, int64_t f, bool report);

fl_status check_basic(int64_t nc, int64_t nf, const int32_t *fc, const double *nrm) {
    if (!fc || !nrm) return fail(FL_E_INVALID, "face_cells and face_normal must not be NULL");
    if (nc < 1 || nf < 1) return fail(FL_E_INVALID, "n_cells and n_faces must be positive");
    if (nc > (int64_t)std::numeric_limits<int32_t>::max() - 1 || nf > (int64_t)(1 << 30) - 1)
        return fail(FL_E_INVALID, "mesh too large for 32-bit cell and face indices");
    int64_t bad = nf;  // the lowest invalid face
#pragma omp parallel for schedule(static) reduction(min : bad)
    for (int64_t f = 0; f < nf; ++f)
        if (check_face(nc, fc, nrm, f, false) != FL_OK) bad = std::min(bad, f);
    return bad < nf ? check_face(nc, fc, nrm, bad, true) : FL_OK;
}

fl_status check_face(int64_t nc, const int32_t *fc, const double *nrm, int64_t f, bool report) {
    auto err = [&](fl_status st, const std::string &m) { return report ? fail(st, m) : st; };
    const int64_t a = fc[2 * f], b = fc[2 * f + 1];
    if (a == -1) {
        std::ostringstream os;
        os << "face " << f << " has no own cell (a boundary face lists its one cell first, "
              "nbr = -1, with the normal pointing out of the mesh)";
        return err(FL_E_TOPOLOGY, os.str());
    }
    if (a < 0 || a >= nc || (b != -1 && (b < 0 || b >= nc))) {
        std::ostringstream os;
        os << "face " << f << " references a cell outside [0, " << nc << ")";
        return err(FL_E_TOPOLOGY, os.str());
    }
    if (a == b) {
        std::ostringstream os;
        os << "face " << f << " joins cell " << a << " to itself";
        return err(FL_E_TOPOLOGY, os.str());
    }
    const double *n = nrm + 3 * f;
    const double n2 = n[0] * n[0] + n[1] * n[1] + n[2] * n[2];
    if (!std::isfinite(n2) || std::fabs(n2 - 1.0) > kNormTol) {
        std::ostringstream os;
        os << "face " << f << " normal is not a finite unit vector";
        return err(FL_E_INVALID, os.str());
    }
    return FL_OK;
}

// Cell c's faces sorted by the cell beyond them; returns the index i > 0 of the first pair of
// faces (i - 1, i) that join c to the same cell, or 0.
size_t duplicate_at(const int32_t *fc, const Csr &cs, int64_t c,
                    std::vector<std::pair<int32_t, int32_t>> &nb) {
    nb.clear();
    for (int64_t p = cs.ptr[c]; p < cs.ptr[c + 1]; ++p)
        if (other(fc, cs.idx[p], c) >= 0) nb.emplace_back(other(fc, cs.idx[p], c), cs.idx[p]);
    std::sort(nb.begin(), nb.end());
    for (size_t i = 1; i < nb.size(); ++i)
        if (nb[i].first == nb[i - 1].first) return i;
    return 0;
}

fl_status check_duplicates(int64_t nc, const int32_t *fc, const Csr &cs) {
    int64_t bad = nc;  // the lowest cell with two faces to one neighbour
#pragma omp parallel reduction(min : bad)
    {
        std::vector<std::pair<int32_t, int32_t>> nb;
#pragma omp for schedule(static)
        for (int64_t c = 0; c < nc; ++c)
            if (duplicate_at(fc, cs, c, nb)) bad = std::min(bad, c);
    }
    if (bad == nc) return FL_OK;
    std::vector<std::pair<int32_t, int32_t>> nb;
    const size_t i = duplicate_at(fc, cs, bad, nb);
    std::ostringstream os;
    os << "faces " << nb[i - 1].second << " and " << nb[i].second << " both join cells " << bad
       << " and " << nb[i].first << " (a periodic side shorter than 3 cells?)";
    return fail(FL_E_TOPOLOGY, os.str());
}

// Weight of face j of cell C for face f with flow sign s: s (n_f . t_j), t_j = n_j oriented into C.
inline double projection(const int32_t *fc, const double *nrm, int64_t f, int64_t j, int64_t C,
                         double s) {
    const double *a = nrm + 3 * f, *b = nrm + 3 * j;
    const double t = fc[2 * j + 1] == C ? 1.0 : -1.0;
    return s * (t * (a[0] * b[0] + a[1] * b[1] + a[2] * b[2]));
}

// far[2f + side], opp[2f + side]: side 0 is C = own, side 1 is C = nbr.  Returns true when every
// side has exactly one projected face, with weight exactly 1 and every other weight exactly 0
// (axis-aligned hexahedra, quadrilaterals, lines in any numbering and orientation:
// d_U = theta_C - theta_U); otherwise far and opp are left at -1.  No tolerance: a mesh whose
// normals are off the axes by any amount keeps all its nonzero weights (side_lists), as the
// upstream difference sums them.
bool far_upwind(int64_t nf, const int32_t *fc, const double *nrm, const Csr &cs,
                std::vector<int32_t> &far, std::vector<int32_t> &opp) {
    far.assign(2 * nf, -1);
    opp.assign(2 * nf, -1);
    bool ok = true;
#pragma omp parallel for schedule(static) reduction(&& : ok)
    for (int64_t f = 0; f < nf; ++f) {
        for (int side = 0; side < 2 && ok; ++side) {
            const int64_t C = fc[2 * f + side];
            const double s = side == 0 ? 1.0 : -1.0;
            int count = 0;
            int64_t jj = -1;
            double ww = 0.0;
            for (int64_t p = cs.ptr[C]; p < cs.ptr[C + 1]; ++p) {
                const int64_t j = cs.idx[p];
                if (j == f) continue;
                const double w = projection(fc, nrm, f, j, C, s);
                if (w != 0.0) {
                    ++count;
                    jj = j;
                    ww = w;
                }
            }
            if (count != 1 || ww != 1.0) {
                ok = false;
                continue;
            }
            far[2 * f + side] = other(fc, jj, C);
            opp[2 * f + side] = (int32_t)jj;
        }
    }
    if (!ok) {
        far.assign(2 * nf, -1);
        opp.assign(2 * nf, -1);
    }
    return ok;
}

// General cells: for every face side, the cells beyond the other faces of C with their nonzero
// weights (the nonzeros of row f of S_{C->F}, T_{C->F} on that side), in C's face order:
// d_U = sum_j w_j (theta_C - theta_j).  With face distances each weight is scaled by d_f / d_j
// (Algorithm UNS's division of each projected difference by the distance across its face, and
// of the face difference by d_f).  Beyond a boundary face j lies the exterior: entry ~j.
// The exterior side of a boundary face (C = the exterior) has no entries: d_U = 0.
bool side_lists(int64_t nf, const int32_t *fc, const double *nrm, const std::vector<double> &dist,
                const Csr &cs, HostTables &t) {
    t.side_ptr.assign(2 * nf + 1, 0);
    t.side_cell.clear();
    t.side_w.clear();
    for (int64_t f = 0; f < nf; ++f)
        for (int side = 0; side < 2; ++side) {
            const int64_t C = fc[2 * f + side];
            const double s = side == 0 ? 1.0 : -1.0;
            for (int64_t p = C >= 0 ? cs.ptr[C] : 0; C >= 0 && p < cs.ptr[C + 1]; ++p) {
                const int64_t j = cs.idx[p];
                if (j == f) continue;
                const double w = projection(fc, nrm, f, j, C, s);
                if (w != 0.0) {
                    const int64_t o = other(fc, j, C);
                    t.side_cell.push_back(o >= 0 ? (int32_t)o : ~(int32_t)j);
                    t.side_w.push_back(dist.empty() ? w : w * (dist[f] / dist[j]));
                }
            }
            if (t.side_cell.size() > (size_t)INT32_MAX) return false;
            t.side_ptr[2 * f + side + 1] = (int32_t)t.side_cell.size();
        }
    return true;
}

// Breadth-first order of the cells (from a pseudo-peripheral start), one component after the
// other.  Returns new_of_old.
std::vector<int32_t> bfs_numbering(int64_t nc, const int32_t *fc, const Csr &cs) {
    auto bfs = [&](int64_t start, std::vector<int32_t> &order) {
        std::vector<char> seen(nc, 0);
        order.clear();
        order.reserve(nc);
        int64_t next_unseen = 0;
        int64_t s = start;
        while ((int64_t)order.size() < nc) {
            if (seen[s]) {
                while (seen[next_unseen]) ++next_unseen;
                s = next_unseen;
            }
            size_t head = order.size();
            order.push_back((int32_t)s);
            seen[s] = 1;
            while (head < order.size()) {
                int64_t c = order[head++];
                for (int64_t p = cs.ptr[c]; p < cs.ptr[c + 1]; ++p) {
                    int64_t o = other(fc, cs.idx[p], c);
                    if (o >= 0 && !seen[o]) {
                        seen[o] = 1;
                        order.push_back((int32_t)o);
                    }
                }
            }
        }
    };
    std::vector<int32_t> order;
    bfs(0, order);
    int64_t start = order.back();
    bfs(start, order);
    std::vector<int32_t> new_of_old(nc);
    for (int64_t i = 0; i < nc; ++i) new_of_old[order[i]] = (int32_t)i;
    return new_of_old;
}

// Space-filling-curve order.  Cell positions are recovered by a breadth-first walk that steps by
// the unit face normal across every face (+n_f from own to nbr): on hexahedral, quadrilateral
// and line meshes this gives the integer lattice coordinates of every cell (a periodic mesh is
// cut open opposite the root).  Cells are then sorted by the Morton (bit-interleaved) code of
// their coordinates, so any run of consecutive cells is a compact block of the mesh and the
// cells a workgroup gathers from lie in it or in the blocks next to it.  Returns new_of_old.
std::vector<int32_t> curve_numbering(int64_t nc, int64_t nf, const int32_t *fc,
                                     const double *nrm, const Csr &cs) {
    // The walk runs level by level on all cores and visits the cells in exactly the order of a
    // serial first-in-first-out walk: a cell's parent is its neighbour of the previous level
    // that comes first in that order (smallest (queue position, face position) claim), and each
    // cell of a level emits the children it won in its face order.
    constexpr uint64_t kUnseen = ~0ULL, kDone = 0;  // claims are 1 + q * D + p
    int64_t D = 1;
    for (int64_t c = 0; c < nc; ++c) D = std::max<int64_t>(D, cs.ptr[c + 1] - cs.ptr[c] + 1);
    std::vector<double> pos(3 * nc, 0.0);
    std::vector<uint64_t> claim(nc, kUnseen);
    std::vector<int32_t> frontier, next;
    std::vector<int64_t> cnt;
    double lo[3] = {0, 0, 0};
    int64_t next_unseen = 0, found = 0;
    double comp_shift = 0.0;  // separate components along x
    while (found < nc) {
        while (claim[next_unseen] != kUnseen) ++next_unseen;
        const int64_t root = next_unseen;
        claim[root] = kDone;
        pos[3 * root] = comp_shift;
        ++found;
        double hi_x = comp_shift;
        frontier.assign(1, (int32_t)root);
        while (!frontier.empty()) {
            const int64_t nq = (int64_t)frontier.size();
#pragma omp parallel for schedule(static)
            for (int64_t q = 0; q < nq; ++q) {
                const int64_t c = frontier[q];
                for (int64_t p = cs.ptr[c]; p < cs.ptr[c + 1]; ++p) {
                    const int64_t o = other(fc, cs.idx[p], c);
                    if (o < 0) continue;
                    const uint64_t key = 1 + (uint64_t)q * D + (uint64_t)(p - cs.ptr[c]);
                    uint64_t cur = __atomic_load_n(&claim[o], __ATOMIC_RELAXED);
                    while (key < cur && !__atomic_compare_exchange_n(&claim[o], &cur, key, true,
                                                                     __ATOMIC_RELAXED,
                                                                     __ATOMIC_RELAXED)) {
                    }
                }
            }
            cnt.assign(nq + 1, 0);
#pragma omp parallel for schedule(static)
            for (int64_t q = 0; q < nq; ++q) {
                const int64_t c = frontier[q];
                int64_t k = 0;
                for (int64_t p = cs.ptr[c]; p < cs.ptr[c + 1]; ++p) {
                    const int64_t o = other(fc, cs.idx[p], c);
                    k += o >= 0 && claim[o] == 1 + (uint64_t)q * D + (uint64_t)(p - cs.ptr[c]);
                }
                cnt[q + 1] = k;
            }
            for (int64_t q = 0; q < nq; ++q) cnt[q + 1] += cnt[q];
            next.resize(cnt[nq]);
#pragma omp parallel for schedule(static) reduction(max : hi_x)
            for (int64_t q = 0; q < nq; ++q) {
                const int64_t c = frontier[q];
                int64_t at = cnt[q];
                for (int64_t p = cs.ptr[c]; p < cs.ptr[c + 1]; ++p) {
                    const int64_t f = cs.idx[p];
                    const int64_t o = other(fc, f, c);
                    if (o < 0 || claim[o] != 1 + (uint64_t)q * D + (uint64_t)(p - cs.ptr[c]))
                        continue;
                    const double s = fc[2 * f] == c ? 1.0 : -1.0;
                    for (int d = 0; d < 3; ++d) pos[3 * o + d] = pos[3 * c + d] + s * nrm[3 * f + d];
                    hi_x = std::max(hi_x, pos[3 * o]);
                    next[at++] = (int32_t)o;
                }
            }
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < (int64_t)next.size(); ++i) claim[next[i]] = kDone;
            found += (int64_t)next.size();
            frontier.swap(next);
        }
        comp_shift = hi_x + 2.0;
    }
    double lo0 = 0.0, lo1 = 0.0, lo2 = 0.0;
#pragma omp parallel for schedule(static) reduction(min : lo0, lo1, lo2)
    for (int64_t c = 0; c < nc; ++c) {
        lo0 = std::min(lo0, pos[3 * c]);
        lo1 = std::min(lo1, pos[3 * c + 1]);
        lo2 = std::min(lo2, pos[3 * c + 2]);
    }
    lo[0] = lo0;
    lo[1] = lo1;
    lo[2] = lo2;
    auto spread = [](uint64_t v) {  // 21 bits -> every third bit
        v &= 0x1fffff;
        v = (v | v << 32) & 0x1f00000000ffffULL;
        v = (v | v << 16) & 0x1f0000ff0000ffULL;
        v = (v | v << 8) & 0x100f00f00f00f00fULL;
        v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
        v = (v | v << 2) & 0x1249249249249249ULL;
        return v;
    };
    // On a periodic lattice the walk reaches the cells half a period from the root from both
    // sides, so that plane is split between the two ends of the coordinate range (which cell
    // lands where depends on the face order), and the tiles along it are ragged.  A face whose
    // step disagrees with its cells' positions crosses that cut; where every such face spans
    // the same whole number P of cells along axis d, the coordinates are folded modulo P.
    int64_t pmn[3] = {INT64_MAX, INT64_MAX, INT64_MAX}, pmx[3] = {0, 0, 0};
    int odd[3] = {0, 0, 0};
#pragma omp parallel for schedule(static) reduction(min : pmn[:3]) reduction(max : pmx[:3], odd[:3])
    for (int64_t f = 0; f < nf; ++f) {
        const int64_t a = fc[2 * f], b = fc[2 * f + 1];
        for (int d = 0; d < 3 && b >= 0; ++d) {
            const double gap = std::fabs(pos[3 * a + d] + nrm[3 * f + d] - pos[3 * b + d]);
            if (gap <= 0.5) continue;
            const int64_t p = std::llround(gap);
            pmn[d] = std::min(pmn[d], p);
            pmx[d] = std::max(pmx[d], p);
            odd[d] = std::max(odd[d], std::fabs(gap - (double)p) > 1e-6 ? 1 : 0);
        }
    }
    int64_t period[3];
    for (int d = 0; d < 3; ++d)
        period[d] = (!odd[d] && pmn[d] == pmx[d] && pmn[d] >= 3) ? pmn[d] : 0;
    std::vector<std::pair<uint64_t, int32_t>> key(nc);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        uint64_t q[3];
        for (int d = 0; d < 3; ++d) {
            const int64_t v = std::llround(pos[3 * c + d] - lo[d]);
            q[d] = (uint64_t)(period[d] ? v % period[d] : v);
        }
        key[c] = {spread(q[0]) | spread(q[1]) << 1 | spread(q[2]) << 2, (int32_t)c};
    }
    __gnu_parallel::sort(key.begin(), key.end());  // keys unique (cell index)
    std::vector<int32_t> new_of_old(nc);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nc; ++i) new_of_old[key[i].second] = (int32_t)i;
    return new_of_old;
}

// Faces sorted by (lower, higher) new cell index.
std::vector<int32_t> face_numbering(int64_t nc, int64_t nf, const int32_t *fc,
                                    const std::vector<int32_t> &cnew) {
    std::vector<int64_t> cnt(nc + 1, 0);
    std::vector<int32_t> lo(nf), hi(nf);
    int64_t *cp = cnt.data();
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < nf; ++f) {
        // a boundary face sorts with its one cell, after that cell's interior faces
        int32_t a = cnew[fc[2 * f]], b = fc[2 * f + 1] >= 0 ? cnew[fc[2 * f + 1]] : (int32_t)nc;
        if (b == (int32_t)nc) {
            lo[f] = a;
            hi[f] = b;
#pragma omp atomic
            cp[lo[f] + 1]++;
            continue;
        }
        lo[f] = std::min(a, b);
        hi[f] = std::max(a, b);
#pragma omp atomic
        cp[lo[f] + 1]++;
    }
    for (int64_t i = 0; i < nc; ++i) cnt[i + 1] += cnt[i];
    std::vector<int32_t> bucket(nf);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    int64_t *fp = fill.data();
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < nf; ++f) {
        int64_t at;
#pragma omp atomic capture
        at = fp[lo[f]]++;
        bucket[at] = (int32_t)f;
    }
    // (hi, f) is unique within a bucket: the order does not depend on how it was filled
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c)
        std::sort(bucket.begin() + cnt[c], bucket.begin() + cnt[c + 1],
                  [&](int32_t x, int32_t y) { return hi[x] < hi[y] || (hi[x] == hi[y] && x < y); });
    std::vector<int32_t> fnew(nf);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < nf; ++i) fnew[bucket[i]] = (int32_t)i;
    return fnew;
}

// Each face is the "forward" face of exactly one of its two cells, and every cell has exactly one
// forward face in each of its opposite-face pairs, so that per-face quantities can be kept in a
// cell-slot layout of P entries per cell (the adjoint's face-velocity cotangent).  First rule:
// face f is forward for the cell it points out of along a lexicographically positive direction
// (own where n_f is lexicographically positive, else nbr).  Opposite faces with exactly opposite
// outward normals (lattice meshes) then split one forward, one backward.  Where that fails for
// some pair, the chains of opposite faces (cell -> face -> next cell -> its opposite face ...) are
// walked and each is oriented along its walk.  Returns fwd[f] = the cell whose forward face f is,
// or an empty vector if no such orientation was found.
std::vector<int32_t> forward_cells(int64_t nc, int64_t nf, const int32_t *fc, const double *nrm,
                                   const Csr &cs, const std::vector<int32_t> &opp) {
    auto side_of = [&](int64_t f, int64_t c) { return fc[2 * f] == c ? 0 : 1; };
    std::vector<int32_t> fwd(nf);
#pragma omp parallel for schedule(static)
    for (int64_t f = 0; f < nf; ++f) {
        const double *n = nrm + 3 * f;
        const bool pos = n[0] > 0.0 || (n[0] == 0.0 && (n[1] > 0.0 || (n[1] == 0.0 && n[2] > 0.0)));
        fwd[f] = pos ? fc[2 * f] : fc[2 * f + 1];
    }
    auto valid = [&]() {
        bool ok = true;
#pragma omp parallel for schedule(static) reduction(&& : ok)
        for (int64_t c = 0; c < nc; ++c)
            for (int64_t p = cs.ptr[c]; p < cs.ptr[c + 1]; ++p) {
                const int64_t f = cs.idx[p], g = opp[2 * f + side_of(f, c)];
                if ((fwd[f] == c) == (fwd[g] == c)) ok = false;
            }
        return ok;
    };
    if (valid()) return fwd;
    // chain walk: from face f0 leaving cell c, the next face is the one of the next cell opposite
    // to the face it was entered by
    std::vector<char> seen(nf, 0);
    for (int64_t f0 = 0; f0 < nf; ++f0) {
        if (seen[f0]) continue;
        int64_t f = f0, c = fc[2 * f0];
        while (!seen[f]) {
            seen[f] = 1;
            fwd[f] = (int32_t)c;
            c = other(fc, f, c);
            f = opp[2 * f + side_of(f, c)];
        }
    }
    if (valid()) return fwd;
    return std::vector<int32_t>();
}

void build_slots(HostTables &t, const Csr &cs, const std::vector<int32_t> &opp) {
    t.pairs = 0;
    // the fused kernel is instantiated for 1, 2 and 3 pairs (lines, quadrilaterals, hexahedra)
    if (!t.uniform_degree || t.max_degree < 2 || (t.max_degree & 1) || t.max_degree > 6) return;
    const int64_t nc = t.nc;
    const int32_t *fc = t.fc.data();
    auto side_of = [&](int64_t f, int64_t c) { return fc[2 * f] == c ? 0 : 1; };
    // opposite faces must pair up: opp(c, opp(c, f)) == f
    bool paired = true;
#pragma omp parallel for schedule(static) reduction(&& : paired)
    for (int64_t c = 0; c < nc; ++c)
        for (int64_t p = cs.ptr[c]; p < cs.ptr[c + 1]; ++p) {
            int64_t f = cs.idx[p];
            int64_t j = opp[2 * f + side_of(f, c)];
            if (opp[2 * j + side_of(j, c)] != f) paired = false;
        }
    if (!paired) return;
    const std::vector<int32_t> fwd = forward_cells(nc, t.nf, fc, t.nrm.data(), cs, opp);
    t.forward_slots = !fwd.empty();
    const int K = t.max_degree, P = K / 2;
    t.slot_face.assign((size_t)K * nc, 0);
    t.slot_nbr.assign((size_t)K * nc, 0);
    t.slot_far.assign((size_t)K * nc, 0);
    t.slot_rev.assign((size_t)K * nc, 0);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        int32_t slots[6];
        int q = 0;
        for (int64_t p = cs.ptr[c]; p < cs.ptr[c + 1]; ++p) {
            int32_t f = cs.idx[p];
            bool placed = false;
            for (int k = 0; k < q; ++k) placed |= (slots[k] == f);
            if (placed) continue;
            const int32_t g = opp[2 * f + side_of(f, c)];
            // slot 2p: the pair's forward face (where the orientation was found)
            const bool swap = t.forward_slots && fwd[g] == c;
            slots[q++] = swap ? g : f;
            slots[q++] = swap ? f : g;
        }
        // pairs in the order of the axis their forward face's normal is closest to, where that
        // axis differs between the cell's pairs (lattice meshes: pair p is axis p)
        if (t.forward_slots) {
            int key[3] = {0, 0, 0};
            bool distinct = true;
            for (int p = 0; p < K / 2; ++p) {
                const double *n = t.nrm.data() + 3 * (int64_t)slots[2 * p];
                const double ax = std::fabs(n[0]), ay = std::fabs(n[1]), az = std::fabs(n[2]);
                key[p] = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
                for (int r = 0; r < p; ++r) distinct &= key[r] != key[p];
            }
            if (distinct)
                for (int p = 1; p < K / 2; ++p)  // insertion sort of at most three pairs
                    for (int r = p; r > 0 && key[r - 1] > key[r]; --r) {
                        std::swap(key[r - 1], key[r]);
                        std::swap(slots[2 * r - 2], slots[2 * r]);
                        std::swap(slots[2 * r - 1], slots[2 * r + 1]);
                    }
        }
        for (int k = 0; k < K; ++k) {
            int32_t f = slots[k];
            int own_side = side_of(f, c) == 0;
            int32_t n = other(fc, f, c);
            size_t at = (size_t)k * nc + c;
            t.slot_face[at] = (uint32_t)f | (own_side ? 0x80000000u : 0u);
            t.slot_nbr[at] = n;
            // far-upwind of f when the flow runs from n into c: on n's side
            t.slot_far[at] = t.far[2 * f + (own_side ? 1 : 0)];
            int32_t rf = opp[2 * f + (own_side ? 1 : 0)];  // face of n opposite to f
            t.slot_rev[at] = (uint32_t)rf | (fc[2 * rf] == n ? 0x80000000u : 0u);
        }
    }
    t.pairs = P;
    // aligned: the neighbour across slot k of every cell sees the shared face in its slot k ^ 1
    bool aligned = t.forward_slots;
    if (aligned) {
#pragma omp parallel for schedule(static) reduction(&& : aligned)
        for (int64_t c = 0; c < nc; ++c)
            for (int k = 0; k < K; ++k) {
                const size_t at = (size_t)k * nc + c;
                const int64_t n = t.slot_nbr[at];
                if ((t.slot_face[(size_t)(k ^ 1) * nc + n] & 0x7fffffffu) !=
                    (t.slot_face[at] & 0x7fffffffu))
                    aligned = false;
            }
    }
    t.aligned_slots = aligned;
}

// The compact forward-stage tables (see HostTables): built from the local slot words where they
// describe them exactly, left empty otherwise.
void build_compact(HostTables &t) {
    const int64_t nc = t.nc, P = t.pairs, K = 2 * P;
    const int64_t ntiles = (nc + kTileCells - 1) / kTileCells;
    if (nc >= (int64_t(1) << 30)) return;
    std::vector<uint16_t> next(t.halo.size(), 0xffff);
    bool ok = true;
#pragma omp parallel for schedule(dynamic, 64) reduction(&& : ok)
    for (int64_t tile = 0; tile < ntiles; ++tile) {
        const int64_t c0 = tile * kTileCells, c1 = std::min(nc, c0 + kTileCells);
        const int64_t h0 = t.halo_ptr[tile];
        for (int64_t k = 0; k < K && ok; ++k)
            for (int64_t c = c0; c < c1; ++c) {
                const uint32_t w = t.slot_local[k * nc + c];
                const uint32_t n = w & 0xffffu, g = w >> 16;
                if (n < (uint32_t)kTileCells) {
                    // the far cell must be the tile neighbour's own neighbour across slot k
                    if ((t.slot_local[k * nc + c0 + n] & 0xffffu) != g) ok = false;
                } else {
                    uint16_t &e = next[h0 + n - kTileCells];
                    if (e == 0xffff) e = (uint16_t)g;
                    else if (e != g) ok = false;
                }
            }
    }
    if (!ok) return;
    t.slot_nb.resize((size_t)P * nc);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c)
        for (int64_t p = 0; p < P; ++p)
            t.slot_nb[p * nc + c] = (t.slot_local[2 * p * nc + c] & 0xffffu) |
                                    (t.slot_local[(2 * p + 1) * nc + c] & 0xffffu) << 16;
    t.halo_pk.resize(t.halo.size());
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)t.halo.size(); ++i)
        t.halo_pk[i] = (int32_t)((uint32_t)t.halo[i] | (uint32_t)t.halo_pair[i] << 30);
    t.halo_next.swap(next);
}

// Tile halos for the LDS-staged fused stage: for each run of kTileCells consecutive cells, the
// sorted list of cells outside the run that its slots name (neighbours and far-upwind cells),
// and every slot's neighbour and far cell as local indices into [tile cells | halo].
void build_tiles(HostTables &t) {
    t.max_halo = -1;
    if (t.pairs < 1) return;
    const int64_t nc = t.nc, K = 2 * t.pairs;
    const int64_t ntiles = (nc + kTileCells - 1) / kTileCells;
    // On meshes with aligned slots a halo entry is a (cell, pair) reference: the cell is reached
    // from the tile along the axis of that pair (as the neighbour or the far cell of a slot of
    // that pair), and the stages that read one rate per face stage that cell's forward rate of
    // that pair beside its values.  A cell reached along two axes (a tile that is not a brick)
    // then appears twice.  Entries are ordered by the stages that need their rate: first those
    // reached as the neighbour across a backward slot (the forward stage and the adjoint need
    // them), then those reached as the neighbour across a forward slot or as the far cell of a
    // backward slot (the adjoint needs them), then the rest (far cells of forward slots: no
    // rate needed); halo_nrate[2 tile + 0 / 1] counts the first group / the first two.
    const bool by_pair = t.aligned_slots;
    std::vector<int32_t> ptr(ntiles + 1, 0), halo, nrate(by_pair ? 2 * ntiles : 0, 0);
    std::vector<uint8_t> halo_pair;
    std::vector<uint32_t> local((size_t)K * nc, 0);
    std::vector<std::vector<int64_t>> tile_refs(ntiles);
    int32_t max_halo = 0, max_nrate = 0, max_nrate0 = 0;
    bool fits = true;
#pragma omp parallel for schedule(dynamic, 64) reduction(max : max_halo, max_nrate, max_nrate0) \
    reduction(&& : fits)
    for (int64_t tile = 0; tile < ntiles; ++tile) {
        const int64_t c0 = tile * kTileCells, c1 = std::min(nc, c0 + kTileCells);
        // (role << 60 | cell << 2 | pair) while collecting; role 0, 1, 2 as above
        std::vector<int64_t> keyed;
        for (int64_t k = 0; k < K; ++k) {
            const int64_t pk = by_pair ? (k >> 1) : 0;
            const int64_t rn = (k & 1) ? 0 : 1, rg = (k & 1) ? 1 : 2;
            for (int64_t c = c0; c < c1; ++c) {
                const int64_t n = t.slot_nbr[k * nc + c], g = t.slot_far[k * nc + c];
                if (n < c0 || n >= c1) keyed.push_back((by_pair ? rn : 0) << 60 | n << 2 | pk);
                if (g < c0 || g >= c1) keyed.push_back((by_pair ? rg : 0) << 60 | g << 2 | pk);
            }
        }
        // one entry per (cell, pair) with its lowest role, ordered by (role, cell, pair)
        const int64_t low = (int64_t(1) << 60) - 1;
        std::sort(keyed.begin(), keyed.end(),
                  [&](int64_t x, int64_t y) { return (x & low) < (y & low) || ((x & low) == (y & low) && x < y); });
        std::vector<int64_t> &refs = tile_refs[tile];
        for (size_t i = 0; i < keyed.size(); ++i)
            if (i == 0 || (keyed[i] & low) != (keyed[i - 1] & low)) refs.push_back(keyed[i]);
        std::sort(refs.begin(), refs.end());
        if (kTileCells + refs.size() > 65535) {  // local indices are 16-bit
            fits = false;
            continue;
        }
        max_halo = std::max<int32_t>(max_halo, (int32_t)refs.size());
        if (by_pair) {
            int32_t n0 = 0, n01 = 0;
            for (int64_t r : refs) {
                n0 += (r >> 60) == 0;
                n01 += (r >> 60) <= 1;
            }
            nrate[2 * tile] = n0;
            nrate[2 * tile + 1] = n01;
            max_nrate = std::max(max_nrate, n01);
            max_nrate0 = std::max(max_nrate0, n0);
        }
        // position of each (cell, pair) in the ordered halo
        std::vector<std::pair<int64_t, int32_t>> pos(refs.size());
        for (size_t i = 0; i < refs.size(); ++i) pos[i] = {refs[i] & low, (int32_t)i};
        std::sort(pos.begin(), pos.end());
        auto loc = [&](int64_t cell, int64_t pk) -> uint32_t {
            if (cell >= c0 && cell < c1) return (uint32_t)(cell - c0);
            const auto it = std::lower_bound(pos.begin(), pos.end(),
                                             std::make_pair(cell << 2 | pk, (int32_t)-1));
            return (uint32_t)(kTileCells + it->second);
        };
        for (int64_t k = 0; k < K; ++k) {
            const int64_t pk = by_pair ? (k >> 1) : 0;
            for (int64_t c = c0; c < c1; ++c)
                local[k * nc + c] = loc(t.slot_nbr[k * nc + c], pk) |
                                    (loc(t.slot_far[k * nc + c], pk) << 16);
        }
    }
    if (!fits) return;
    // the halos one after the other, in tile order
    size_t total = 0;
    for (int64_t tile = 0; tile < ntiles; ++tile) {
        total += tile_refs[tile].size();
        if (total > (size_t)INT32_MAX) return;
        ptr[tile + 1] = (int32_t)total;
    }
    halo.resize(total);
    if (by_pair) halo_pair.resize(total);
    const int64_t low = (int64_t(1) << 60) - 1;
#pragma omp parallel for schedule(static)
    for (int64_t tile = 0; tile < ntiles; ++tile)
        for (size_t i = 0; i < tile_refs[tile].size(); ++i) {
            const int64_t r = tile_refs[tile][i] & low;
            halo[ptr[tile] + i] = (int32_t)(r >> 2);
            if (by_pair) halo_pair[ptr[tile] + i] = (uint8_t)(r & 3);
        }
    t.halo_ptr.swap(ptr);
    t.halo.swap(halo);
    t.halo_pair.swap(halo_pair);
    t.halo_nrate.swap(nrate);
    t.slot_local.swap(local);
    t.max_halo = max_halo;
    t.max_nrate = by_pair ? max_nrate : -1;
    t.max_nrate0 = by_pair ? max_nrate0 : -1;
    if (by_pair) build_compact(t);
}

}  // namespace

fl_status build_host_tables(int64_t nc, int64_t nf, const int32_t *face_cells,
                            const double *face_normal, const double *face_area,
                            const double *cell_volume, const double *face_dist, int reorder,
                            HostTables &t) {
    Progress progress;
    fl_status st = check_basic(nc, nf, face_cells, face_normal);
    if (st != FL_OK) return st;
    if (face_area)
        for (int64_t f = 0; f < nf; ++f)
            if (!(face_area[f] > 0.0) || !std::isfinite(face_area[f]))
                return fail(FL_E_INVALID, "face areas must be finite and positive");
    if (cell_volume)
        for (int64_t c = 0; c < nc; ++c)
            if (!(cell_volume[c] > 0.0) || !std::isfinite(cell_volume[c]))
                return fail(FL_E_INVALID, "cell volumes must be finite and positive");
    if (face_dist)
        for (int64_t f = 0; f < nf; ++f)
            if (!(face_dist[f] > 0.0) || !std::isfinite(face_dist[f]))
                return fail(FL_E_INVALID, "face distances must be finite and positive");

    t = HostTables();
    t.nc = nc;
    t.nf = nf;
    t.fc.assign(face_cells, face_cells + 2 * nf);
    t.nrm.assign(face_normal, face_normal + 3 * nf);
    std::vector<double> area, vol, dist;
    if (face_area) area.assign(face_area, face_area + nf);
    if (cell_volume) vol.assign(cell_volume, cell_volume + nc);
    // equal distances leave every ratio d_f / d_j at 1: the unweighted tables
    if (face_dist)
        for (int64_t f = 1; f < nf && dist.empty(); ++f)
            if (face_dist[f] != face_dist[0]) dist.assign(face_dist, face_dist + nf);

    Csr cs = cell_faces(nc, nf, t.fc.data());
    st = check_duplicates(nc, t.fc.data(), cs);
    if (st != FL_OK) return st;
    progress("validated", nc);

    if (reorder) {
        std::vector<int32_t> cnew = reorder == REORDER_BFS
                                        ? bfs_numbering(nc, t.fc.data(), cs)
                                        : curve_numbering(nc, nf, t.fc.data(), t.nrm.data(), cs);
        progress("cells renumbered", nc);
        std::vector<int32_t> fnew = face_numbering(nc, nf, t.fc.data(), cnew);
        std::vector<int32_t> fc2(2 * nf);
        std::vector<double> nrm2(3 * nf);
#pragma omp parallel for schedule(static)
        for (int64_t f = 0; f < nf; ++f) {
            int64_t g = fnew[f];
            fc2[2 * g] = cnew[t.fc[2 * f]];
            fc2[2 * g + 1] = t.fc[2 * f + 1] >= 0 ? cnew[t.fc[2 * f + 1]] : -1;
            std::memcpy(&nrm2[3 * g], &t.nrm[3 * f], 3 * sizeof(double));
        }
        if (!area.empty()) {
            std::vector<double> a2(nf);
#pragma omp parallel for schedule(static)
            for (int64_t f = 0; f < nf; ++f) a2[fnew[f]] = area[f];
            area.swap(a2);
        }
        if (!dist.empty()) {
            std::vector<double> d2(nf);
#pragma omp parallel for schedule(static)
            for (int64_t f = 0; f < nf; ++f) d2[fnew[f]] = dist[f];
            dist.swap(d2);
        }
        if (!vol.empty()) {
            std::vector<double> v2(nc);
#pragma omp parallel for schedule(static)
            for (int64_t c = 0; c < nc; ++c) v2[cnew[c]] = vol[c];
            vol.swap(v2);
        }
        t.fc.swap(fc2);
        t.nrm.swap(nrm2);
        t.cell_perm.swap(cnew);
        t.face_perm.swap(fnew);
        cs = cell_faces(nc, nf, t.fc.data());
        progress("faces renumbered", nc);
    }

    // uniform area / volume are kept as one scalar
    t.uni_area = true;
    t.area0 = area.empty() ? 1.0 : area[0];
    for (double a : area) t.uni_area &= (a == t.area0);
    if (!t.uni_area) t.area.swap(area);
    t.uni_vol = true;
    t.vol0 = vol.empty() ? 1.0 : vol[0];
    for (double v : vol) t.uni_vol &= (v == t.vol0);
    if (!t.uni_vol) t.vol.swap(vol);

    std::vector<int32_t> opp;
    t.n_boundary = 0;
    for (int64_t f = 0; f < nf; ++f) t.n_boundary += t.fc[2 * f + 1] < 0;
    // a mesh with boundary faces runs the general face path: the exterior beyond a boundary
    // face has no far-upwind cell and no opposite face; so does a mesh with unequal face
    // distances (its side weights carry the distance ratios)
    t.dist_weighted = !dist.empty();
    t.general = t.n_boundary > 0 || t.dist_weighted ||
                !far_upwind(nf, t.fc.data(), t.nrm.data(), cs, t.far, opp);
    if (t.n_boundary > 0 || t.dist_weighted) {
        t.far.assign(2 * nf, -1);
        opp.assign(2 * nf, -1);
    }
    if (t.general && !side_lists(nf, t.fc.data(), t.nrm.data(), dist, cs, t))
        return fail(FL_E_UNSUPPORTED, "too many projected faces for 32-bit side lists");
    if (t.general) {
        // the transpose of the side lists (cells beyond a boundary face are not cells)
        t.rev_ptr.assign(nc + 1, 0);
        for (int32_t c : t.side_cell)
            if (c >= 0) t.rev_ptr[c + 1]++;
        for (int64_t c = 0; c < nc; ++c) t.rev_ptr[c + 1] += t.rev_ptr[c];
        t.rev_side.resize(t.rev_ptr[nc]);
        t.rev_w.resize(t.rev_ptr[nc]);
        std::vector<int32_t> fill(t.rev_ptr.begin(), t.rev_ptr.end() - 1);
        for (int64_t sd = 0; sd < 2 * nf; ++sd)
            for (int32_t p = t.side_ptr[sd]; p < t.side_ptr[sd + 1]; ++p) {
                const int32_t c = t.side_cell[p];
                if (c < 0) continue;
                t.rev_side[fill[c]] = (int32_t)sd;
                t.rev_w[fill[c]++] = t.side_w[p];
            }
    }
    progress("far-upwind cells", nc);

    t.cf_ptr.resize(nc + 1);
    t.cf_idx.resize(cs.idx.size());
    int32_t max_degree = 0;
    int32_t min_degree = std::numeric_limits<int32_t>::max();
    for (int64_t c = 0; c <= nc; ++c) t.cf_ptr[c] = (int32_t)cs.ptr[c];
#pragma omp parallel for schedule(static) reduction(max : max_degree) reduction(min : min_degree)
    for (int64_t c = 0; c < nc; ++c) {
        int32_t d = (int32_t)(cs.ptr[c + 1] - cs.ptr[c]);
        max_degree = std::max(max_degree, d);
        min_degree = std::min(min_degree, d);
        for (int64_t p = cs.ptr[c]; p < cs.ptr[c + 1]; ++p) {
            int32_t f = cs.idx[p];
            t.cf_idx[p] = (t.fc[2 * f + 1] == c) ? f : ~f;
        }
    }
    t.max_degree = max_degree;
    t.uniform_degree = (min_degree == t.max_degree);
    if (!t.general) build_slots(t, cs, opp);
    progress("slot tables", nc);
    build_tiles(t);
    progress("tile tables", nc);
    return FL_OK;
}

}  // namespace fl

// Internal declarations of the flux-limiter library (not part of the C ABI).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fluxlim.h"

namespace fl {

// Thread-local error text behind fl_last_error().
void set_error(const std::string &msg);
fl_status fail(fl_status st, const std::string &msg);

// Host-side tables of a mesh, all in mesh order (see fl_mesh_create).
struct HostTables {
    int64_t nc = 0, nf = 0;
    std::vector<int32_t> fc;        // [F][2] own, nbr
    std::vector<double> nrm;        // [F][3]
    std::vector<double> area;       // [F] (empty if uniform)
    std::vector<double> vol;        // [C] (empty if uniform)
    double area0 = 1.0, vol0 = 1.0; // the uniform values
    bool uni_area = true, uni_vol = true;
    std::vector<int32_t> far;       // [F][2] far-upwind cell for C = own, C = nbr (-1: general)
    // General cells (general = true): per face side (2f + side), the far cells and weights of
    // the upstream difference d_U = sum_j w_j (theta_C - theta_j), CSR over 2F sides.
    bool general = false;
    std::vector<int32_t> side_ptr;   // [2F + 1]
    std::vector<int32_t> side_cell;
    std::vector<double> side_w;
    // Their transpose for the general adjoint: per cell, the face sides whose d_U names it
    // (2f + side) with the weight, in ascending side order.
    std::vector<int32_t> rev_ptr;    // [C + 1]
    std::vector<int32_t> rev_side;
    std::vector<double> rev_w;
    std::vector<int32_t> cf_ptr;    // [C+1]
    std::vector<int32_t> cf_idx;    // signed: f (cell is nbr) or ~f (cell is own), ascending f
    int32_t max_degree = 0;
    bool uniform_degree = false;
    int32_t pairs = 0;              // > 0 iff every cell has 2*pairs faces in opposite pairs
    // Slot 2p of every cell is its forward face of pair p: each face is forward for exactly one
    // of its cells (true for every fused-path mesh where the orientation was found).
    bool forward_slots = false;
    // Every cell's neighbour across its slot k holds the shared face in its slot k ^ 1 (lattice
    // meshes, whose pairs are ordered by axis): a quantity of slot k of that neighbour describes
    // the face beyond it in the same direction.
    bool aligned_slots = false;
    // Fused-path slot tables, structure of arrays [2*pairs][C].
    std::vector<uint32_t> slot_face; // face index | (1u << 31) if the cell is the face's own
    std::vector<int32_t> slot_nbr;   // the other cell of the face
    std::vector<int32_t> slot_far;   // far-upwind cell of the face on the other cell's side
    std::vector<uint32_t> slot_rev;  // face of the other cell opposite to this slot's face
                                     // | (1u << 31) if the other cell is that face's own
    // Tiles of kTileCells consecutive cells for the LDS-staged fused stage (fused path only):
    // tile t stages its own cells and the cells its slots reference outside it (its halo,
    // ascending) in LDS; slot_local[k][c] = local index of n_k | local index of g_k << 16
    // (0 .. kTileCells-1: the tile's own cells; kTileCells + j: halo entry j).
    std::vector<int32_t> halo_ptr;   // [tiles + 1]
    std::vector<int32_t> halo;       // cell indices
    std::vector<uint32_t> slot_local;
    // Aligned slots: the pair along which each halo entry is reached (halo entries are then
    // (cell, pair) references; a cell may appear once per pair).
    std::vector<uint8_t> halo_pair;
    // Aligned slots: per tile, how many leading halo entries the forward-rate stage needs the
    // rate of, and how many the forward-rate adjoint stage does ([2 * tiles]).
    std::vector<int32_t> halo_nrate;
    int32_t max_halo = -1;           // -1: no tile tables (local indices would not fit 16 bits)
    int32_t max_nrate = -1;          // largest halo_nrate[2 tile + 1] (-1: not aligned)
    int32_t max_nrate0 = -1;         // largest halo_nrate[2 tile]
    // Compact forward-stage tables (aligned slots, where the far cell of every slot is the
    // neighbour's neighbour in the same direction and every halo entry reached as a neighbour
    // is reached along one direction; empty otherwise):
    //   slot_nb[p][c]  = local index of the neighbour across slot 2p | across slot 2p+1 << 16;
    //   halo_pk[i]     = halo[i] | halo_pair[i] << 30 (cells < 2^30);
    //   halo_next[i]   = for an entry reached as the neighbour across slot k of a tile cell, the
    //                    local index of the cell beyond it in that direction (0xffff if none).
    std::vector<uint32_t> slot_nb;
    std::vector<int32_t> halo_pk;
    std::vector<uint16_t> halo_next;
    int64_t n_boundary = 0;          // faces with one cell (nbr == -1): general face path only
    bool dist_weighted = false;      // side weights scaled by face distance ratios d_f / d_j
    // Numbering maps user -> mesh (empty = identity).
    std::vector<int32_t> cell_perm, face_perm;
};

constexpr int kTileCells = 256;
// Halo entries per thread whose theta is gathered before the slot loads are issued (two: the
// 512-cell halo of a whole 8x8x4 brick; larger halos take a loop for the rest).  The device
// halo array carries kHaloPad extra zeros (cell 0), so that every tile, also one with an empty
// halo at the end, has a first entry to read.
constexpr int kHaloAhead = 2;
constexpr int kHaloPad = 1;

enum { REORDER_NONE = 0, REORDER_CURVE = 1, REORDER_BFS = 2 };

// Validates and builds every table; returns FL_OK or an error (message set).
fl_status build_host_tables(int64_t nc, int64_t nf, const int32_t *face_cells,
                            const double *face_normal, const double *face_area,
                            const double *cell_volume, const double *face_dist, int reorder,
                            HostTables &t);

}  // namespace fl

// Device-side mesh (opaque to users).
struct fl_mesh {
    fl::HostTables h;
    int device = -1;
    int path = FL_PATH_FACE_CELL;
    bool reordered = false;
    // device tables
    int32_t *d_fc4 = nullptr;      // [F][4] own, nbr, far_own, far_nbr
    int32_t *d_cf_ptr = nullptr;   // [C+1] (null when every cell has max_degree faces)
    int32_t *d_cf_idx = nullptr;   // signed face lists
    uint32_t *d_slot_face = nullptr;
    int32_t *d_slot_nbr = nullptr;
    int32_t *d_slot_far = nullptr;
    int32_t *d_side_ptr = nullptr; // general cells: per-side far cells and weights
    int32_t *d_side_cell = nullptr;
    double *d_side_w = nullptr;
    int32_t *d_rev_ptr = nullptr;  // general cells: the transposed side lists
    int32_t *d_rev_side = nullptr;
    double *d_rev_w = nullptr;
    int32_t *d_halo_ptr = nullptr; // LDS-staged stage: tile halo lists and local slot indices
    int32_t *d_halo = nullptr;
    uint32_t *d_slot_local = nullptr;
    uint8_t *d_halo_pair = nullptr;  // [halo entries + pad] pair of each halo entry (aligned slots)
    uint32_t *d_slot_nb = nullptr;   // compact forward-stage tables (HostTables)
    int32_t *d_halo_pk = nullptr;    // [halo entries + pad]
    uint16_t *d_halo_next = nullptr; // [halo entries + pad]
    int32_t *d_halo_nrate = nullptr; // [2 * tiles] halo entries whose rates the stages need
    int32_t *d_adj_fr = nullptr;   // [2P][C][2] LDS adjoint: slot face, the neighbour's face
                                   // opposite it (both with own bits)
    int32_t *d_adj_rec = nullptr;  // [2P][C][4] adjoint: slot face, the neighbour's face opposite
                                   // it (both with own bits), neighbour, far cell
    double *d_area = nullptr;      // [F] if non-uniform
    double *d_vol = nullptr;       // [C] if non-uniform
    int32_t *d_cell_perm = nullptr, *d_face_perm = nullptr;  // user -> mesh
    int64_t device_bytes = 0;
    // caller's inflow values of the boundary faces ([F][inflow_S], device; fl_mesh_set_inflow)
    const double *inflow = nullptr;
    int inflow_S = 0;
};

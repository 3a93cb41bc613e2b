// relres_internal.h -- data layout shared by the host API (relres_host.cpp)
// and the gfx950 kernels (relres_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "relres.h"

namespace relres {

// A list entry packs the caller index of the neighbour (27 bits) and its atom
// type (5 bits), so the force kernel needs no separate type gather.
constexpr int kIdxBits = 27;
constexpr uint32_t kIdxMask = (1u << kIdxBits) - 1u;

// Per-type-pair coefficients of Eq. 20, split into the part carried by the FG
// potential (non-zero on [0, r_s+)) and the part carried by the CG potential
// (non-zero on [0, r_c+), hybrid pairs only).  With delta = r - r_-:
//   FG:  r <  r_s-        u_FG(r)            - f_s-^FG(Dr_s)
//        r in [r_s-,r_s+) f_s-^FG(delta)     - f_s-^FG(Dr_s)
//   CG:  r <  r_s-        gamma_0+^CG        - Gamma_c-      (no force)
//        r in [r_s-,r_s+) f_s+^CG(delta)     - Gamma_c-
//        r in [r_s+,r_c-) u_CG(r)            - Gamma_c-'
//        r in [r_c-,r_c+) f_c-^CG(delta)     - Gamma_c-'
// Summed, the two parts reproduce every case of Eq. 20 with the constants of
// Eq. 19 (Gamma_s+ = Gamma_c- + f_s-^FG(Dr_s), Gamma_s- = Gamma_s+ - gamma_0+).
// Gamma_c-' is Gamma_c- (pair_modify shift yes) or 0 (shift no, which leaves
// Gamma_s+- as they are).  The distances r_s-, r_s+, r_c-, r_c+ belong to the
// type pair when they are set per type.
// LJ terms use  -u'(r)/r = r^-8 (c12 r^-6 - c6),  u(r) = r^-6 (e12 r^-6 - e6)
// with c12 = 48 eps sig^12, c6 = 24 eps sig^6, e12 = 4 eps sig^12, e6 = 4 eps sig^6.
template <typename S>
struct PairCoef {
    S fg_c12, fg_c6, fg_e12, fg_e6;
    S fg_g[5];          // f_s-^FG coefficients gamma_0- .. gamma_4-
    S fg_shift;         // f_s-^FG(Dr_s)
    S cg_c12, cg_c6, cg_e12, cg_e6;
    S sp_g0, sp_g3, sp_g4;  // f_s+^CG: gamma_0+, gamma_3+, gamma_4+ (gamma_1+ = gamma_2+ = 0)
    S cm_g[5];          // f_c-^CG coefficients
    S cm_shift;         // Gamma_c-' (cases 3-4 of Eq. 20)
    S sp_shift;         // Gamma_c- (cases 1-2, inside Gamma_s+-)
};

template <typename S>
struct Cutoffs {
    S rsi, rso, rci, rco;        // r_s-, r_s+, r_c-, r_c+
    S rsi2, rso2, rci2, rco2;    // their squares
};

// Cell grid of one system for one kind of list (atom grid: cells >= r_s+ +
// skin over all atoms; site grid: cells >= r_c+ + skin over hybrid atoms).
struct GeomDev {
    int n[3];                 // cells per axis
    int cell_base;            // global rank of this grid's first cell
    double inv_cell[3];       // n_k / L_k
    double box[3];            // L_k of the system
    double half[3];           // L_k / 2
    int row_base;             // global row of this grid's first member
    int members;
    int wave_base;            // first wave of this grid in the list kernel
    int pad;
    double rl2;               // list radius squared (r_+ + the system's skin)^2
    double half_skin2;        // (the system's skin / 2)^2
};

// All grids of one kind, one per system, concatenated: cells are numbered
// grid after grid (Morton order inside a grid) and member rows follow the
// cells, so the rows of a system are contiguous.
struct GridDev {
    int nsys;
    int ncell;                // cells of all grids
    int members;              // members of all grids
    int cap;                  // row capacity of the padded list
    int waves;                // waves of the list kernel for this kind
    int rows_per_wave;        // consecutive home rows per wave (<= kRowsPerWave)
    const GeomDev* geom;      // [nsys]
    const int* wave_sys;      // [waves] system of each list-kernel wave (nsys > 1; else null)
    const int* cell_sys;      // [ncell] system of each cell
    const int* rank_of_lin;   // [cell_base + local linear index] -> global cell rank
    const int* lin_of_rank;   // [global cell rank] -> local linear index
    const int* nbr;           // ncell x 27 stencil ranks (-1: slot unused after deduplication);
                              // only for stencil 3
    int stencil;              // cells per axis of the list stencil: 3 (cells of at least the
                              // list radius) or 5 (cells of at least half of it)
    int* count;               // per cell (by rank); zero between builds
    int* start;               // ncell + 1 exclusive offsets (by rank)
    int* user_unsorted;       // member caller indices, cell-grouped; with bucket_cap > 0 the
                              // per-cell buckets (ncell x bucket_cap) that k_bin fills
    int bucket_cap;           // > 0: members go straight into per-cell buckets, k_place
                              // places them and the list kernel clears the counts
    int* user;                // member caller indices, cell-grouped, ascending in a cell
    double4* pos;             // wrapped positions of members; w: entry and molecule bits
                              // (member_tag in the kernels)
    int2* meta;               // (type, molecule) of members
    int* row_cell;            // cell rank of each member row
    int* list;                // rows x cap entries
    int* nrow;                // entries per row (true count, may exceed cap)
};

struct TopoDev {
    const int* types;
    const int* mol;
    const int* hybrid;        // per type: 1 if eps_cg > 0
    const int* excl_off;      // CSR (caller indices), symmetrised; may be null
    const int* excl_idx;
    int same_mol;
    int n;
    int max_excl;             // most excluded partners of any atom
    const int* sys;           // system of each atom, or null when there is one system
};

// Build status, in device memory; the host copies it to pinned memory to
// examine it.  Every field but the on-demand statistics only grows, so one
// examination covers every build since the previous one (for instance all
// replays of a captured graph): max_row is written only by rows that outgrew
// their capacity and is never cleared (capacities only grow, past every value
// seen, so max_row > capacity means a build since the last growth
// overflowed); entries and longest are filled on demand by k_list_stats.
struct Status {
    int nonfinite;                  // cumulative count of non-finite positions seen
    int max_row[2];                 // longest overflowing row per grid since creation, 0 if none
    int longest[2];                 // longest row per grid (k_list_stats)
    unsigned moved;                 // cumulative count, over builds, of atoms found more
                                    // than half the skin from their previous-build position
    unsigned long long entries[2];  // entries per grid (k_list_stats)
    unsigned moved_query;           // the same count for relres_moved_atoms
    unsigned pad;
    unsigned ew_failed;             // cumulative count of energy/virial waits that gave up
    unsigned pad2;
};

struct ForceArgs {
    const double* pos;        // caller positions, N x 3
    double box[3];            // box of system 0 (the only one when nsys == 1)
    double inv_box[3];
    int nsys;
    const double* boxes;      // [nsys][6]: L_x, L_y, L_z, 1/L_x, 1/L_y, 1/L_z
    double* row_ew;           // nsys > 1: 8 FP64 partials per row (atom rows, then site
                              // rows), written only by waves across a system boundary
    double* wave_ew;          // nsys > 1: 8 FP64 sums per wave (atom waves, then site waves)
    int* wave_sys;            // ... and the wave's system; -1: across a boundary (rows in
                              // row_ew), -2: no rows of its own
    // atom list rows (all atoms, atom-grid order); record = (caller index,
    // type + 32 system, stored entries, 1 if hybrid)
    int n_arow;
    const int4* a_rec;
    const int* a_list;
    int a_cap;
    // site list rows (hybrid atoms, site-grid order); record = (caller index,
    // type + 32 system, stored entries, atom-list row of the same atom)
    int n_srow;
    const int4* s_rec;
    const int* s_list;
    int s_cap;
    const void* coef32;       // PairCoef<float>[ntypes * ntypes]
    const void* coef64;       // PairCoef<double>[ntypes * ntypes]
    const Cutoffs<float>* pcut32;    // distances per type pair [ntypes * ntypes]
    const Cutoffs<double>* pcut64;
    int ntypes;
    void* forces;             // N x 3 of TF, caller order
    double* energy;           // [nsys][3] or null
    double* virial;           // [nsys][6] or null
    unsigned long long* ew_rec;   // energy/virial records: one per block, then one per group
    unsigned int* epoch;          // launch epoch, advanced by every energy/virial launch
    unsigned int* ew_failed;      // Status::ew_failed, counted by a wait that gave up
    int spin_limit;               // polls of a cross-block wait before it gives up (< 0: at once)
    int wide_batch;               // forces-only launches: 4 entries per lane per batch, not 2
    int blocks_a, blocks_b;   // multiples of 8
    int lanes_a, lanes_b;     // lanes per row (powers of two)
    int log_lanes_a, log_lanes_b;
};

// Launchers (relres_kernels.hip).  All return hipError_t of the launch.
// check_moved: before overwriting wpos, count in st->moved the atoms whose
// position is more than half their system's skin (minimum image) from the
// wpos of the previous build (a comparable previous build exists)
hipError_t launch_bin(int n, const double* pos, TopoDev topo, GridDev* grids_dev, double4* wpos,
                      int2* key_a, int2* key_s, Status* st, bool check_moved, hipStream_t s);
// st->moved_query += atoms of pos more than half their system's skin from wpos
hipError_t launch_moved(int n, const double* pos, TopoDev topo, const GridDev* grids_dev,
                        const double4* wpos, Status* st, hipStream_t s);
// Exclusive scan of the cell counts of both grids (one block per grid, or
// with more than one segment per grid a two-launch scan over all segments
// using seg_tot: scan_segments(ncell_a) + scan_segments(ncell_s) ints)
int scan_segments(int ncell);
hipError_t launch_scan(GridDev* grids_dev, int ngrids, int ncell_a, int ncell_s, int* seg_tot,
                       hipStream_t s);
hipError_t launch_scatter(int n, GridDev* grids_dev, const int2* key_a, const int2* key_s,
                          hipStream_t s);
// members: rows of both grids (picks cells per wave)
hipError_t launch_cellsort(GridDev* grids_dev, int ncell_a, int ncell_total, long long members,
                           const double4* wpos, TopoDev topo, int* user2arow, hipStream_t s);
// Grids of few cells: scan, scatter and cell sort in one launch.  k_bin has
// filed every member into its cell's bucket (GridDev::bucket_cap > 0); each
// block adds up the counts of the cells before its own, then ranks and places
// its cells' members (a cell that outgrew its bucket finds its members in the
// key arrays).  kPlaceMaxCells bounds the cells of both grids together, since
// the count sums are repeated by every block.
constexpr int kPlaceMaxCells = 8192;
hipError_t launch_place(GridDev* grids_dev, int ncell_a, int ncell_s, long long members, int n,
                        const int2* key_a, const int2* key_s, const double4* wpos, TopoDev topo,
                        int* user2arow, hipStream_t s);
// per_wave: one wave per home cell (small cells) instead of one block per cell
// Candidates per lane of the row-group list kernel (2 or 4) for a launch of
// total_waves waves; cand = 2 or 4 forces the value, 0 chooses it.
int list_candidates(int total_waves, int cand);
// stencil_a, stencil_s: 3 or 5 (GridDev::stencil of each grid); the
// block-per-cell kernel only serves two 27-cell stencils
hipError_t launch_lists(GridDev* grids_dev, int ncell_a, int ncell_s, int waves_a, int waves_s,
                        TopoDev topo, const int* user2arow, int4* a_rec, int4* s_rec, Status* st,
                        bool per_wave, int cand, int stencil_a, int stencil_s, hipStream_t s);
// cut64 = {r_s-, r_s+, r_c-, r_c+, and their squares} of every type pair, or
// per_pair: the distances of each type pair come from a.pcut32 / a.pcut64
hipError_t launch_forces(const ForceArgs& a, const double* cut64, bool per_pair, int pair_math,
                         int precision, bool ew, hipStream_t s);
hipError_t launch_list_stats(GridDev* grids_dev, int ngrids, Status* st, hipStream_t s);
// Backward (adjoint) pass: ForceArgs (positions, lists, FP64 table) plus
struct BackArgs {
    ForceArgs f;
    const double* gforce;                 // dJ/dF, N x 3, or NULL
    const double* genergy;                // dJ/dE per system (device, nsys) or NULL
    double* gpos;                         // out: dJ/dx, N x 3
    const PairCoef<double>* cgrad;        // [4][ntypes^2] derivative records
    double* partial;                      // per wave: [ntypes^2][4] parameter sums
};
constexpr int kBackwardTypes = 8;
// waves = wavefronts of the launch; grad_pair receives [4][ntypes][ntypes];
// distances per type pair from b.f.pcut64
hipError_t launch_backward(const BackArgs& b, int waves, double* grad_pair, hipStream_t s);
// per-type gradients [4][nt] from pair gradients [4][nt][nt] and the mixing
// Jacobian [2][nt][nt][6] (relres_backward_types)
hipError_t launch_type_grad(const double* gpair, const double* jac, int nt, double* gtype,
                            hipStream_t s);
hipError_t launch_clear_words(unsigned long long* p, size_t n, hipStream_t s);
// Static scratch of relres_forces_noalloc (relres_kernels.hip): 256 bytes of
// launch epoch, then energy/virial records.  scratch_address() must be called
// with the device current; it returns that device's copy.
constexpr size_t kScratchBytes = RELRES_NOALLOC_SCRATCH_BYTES;
constexpr size_t kScratchEpochBytes = 256;
hipError_t scratch_address(void** out);
hipError_t launch_zero_outputs(double* energy, double* virial, int nsys, hipStream_t s);
// nsys > 1: energy/virial of each system from the wave sums (and the row
// partials of waves across a system boundary)
hipError_t launch_reduce_sys_ew(const GridDev* grids_dev, int ngrids, const ForceArgs& a,
                                double* energy, double* virial, hipStream_t s);

// Bonded terms and scaled 1-4 pairs (relres_md.hip).  Per atom, the terms
// it belongs to: term_ent packs kind (bits 30-31: 0 bond, 1 angle,
// 2 dihedral), the atom's slot in the term (bits 28-29) and the term index.
// One item of an atom's bonded work: a (term, slot) entry or a 1-4 partner.
// Atoms of the term in the term's order (a bond uses i, j; an angle i, j =
// vertex, k; a dihedral i, j, k, l); a 1-4 item has i = the atom, j = the
// partner and par = the pair's type-pair index.  kind -1 marks padding.
struct BondItem {
    int kind;                         // 0 bond, 1 angle, 2 dihedral, 3 1-4 pair, -1 none
    int slot;                         // the atom's place in the term
    int i, j, k, l;
    int par;                          // row of bond_par / angle_par / dih_par, or type pair
    int pad;
};
struct BondedArgs {
    const double* pos;
    double box[3];
    int n;
    const BondItem* items;            // n x slots, atom-major; padded with kind -1
    int slots;                        // items per atom (a power of two)
    const double2* bond_par;          // K, r0
    const double2* angle_par;         // K, theta0
    const double4* dih_par;           // K, n, cos d, sin d
    double scale14;
    const PairCoef<double>* coef64;
    const Cutoffs<double>* pcut64;
    void* forces;                     // N x 3 of the force type; added to
    double* partial;                  // per block: 4 energies, 6 virial; or null
    int log_lanes;                    // lanes per atom = 2^log_lanes (<= slots, <= 32)
};
struct MdArgs;
// Bonded and 1-4 forces added to b.forces; with m, also the half kick of a
// dynamics step and the kinetic partials (m->partial).
hipError_t launch_bonded(const BondedArgs& b, const MdArgs* m, int force_prec, hipStream_t s);
int md_blocks(int n);                 // blocks of the one-thread-per-atom kernels
int bonded_blocks(int n, int log_lanes);   // blocks of the bonded kernel
// out[k] = sum of p1[blk * K + k] over its blocks, then of p2, in block order
hipError_t launch_sum_partials(const double* p1, int n1, const double* p2, int n2, int K,
                               double* out, hipStream_t s);

// Thermostat and integrator state on the device.
struct MdState {
    double xi, eta;                   // thermostat velocity and position
    double K;                         // kinetic energy of the true velocities
    double s2;                        // pending velocity scale (true v = stored v * s2)
    double s_apply;                   // scale the next drift applies to stored v
    double s_last;
    double dt, kT, g, Q;
};
struct MdArgs {
    int n;
    double ftm2v;                     // force / mass -> acceleration
    double* pos;                      // N x 3, updated in place
    double* vel;                      // N x 3, stored velocities
    const void* forces;               // N x 3 of the force type
    const double* mass;
    const double* xref;               // positions at the last list build
    double half_skin2;                // (skin / 2)^2
    unsigned int* stale;              // set when an atom moved more than skin / 2
    double* partial;                  // per block kinetic partial
    MdState* st;
};
// Drift of one step; with scalar != 0 every block first does the scalar work
// between the previous step and this one from st_in (kinetic partials
// m.partial[0..nparts), the thermodynamic row when row != 0) and block 0
// stores the new state in st_out (a different buffer).
hipError_t launch_md_drift(const MdArgs& m, const MdState* st_in, MdState* st_out, int nparts,
                           int scalar, const double* e_nb, const double* w_nb, const double* eb,
                           double* row, int force_prec, hipStream_t s);
hipError_t launch_md_kinetic(const MdArgs& m, hipStream_t s);
// kinetic energy from the partials; second / first thermostat half steps;
// with row, one row of thermodynamic output
hipError_t launch_md_scalar(MdState* st, const double* partial, int nblocks, double ftm2v,
                            int second, int first, const double* e_nb, const double* w_nb,
                            const double* eb, double* row, hipStream_t s);
hipError_t launch_md_finish(const MdArgs& m, hipStream_t s);

// Row record field y: atom type in the low kTypeBits bits, system above.
constexpr int kTypeBits = 5;
constexpr int kRowsPerWave = 16;      // most home rows per wave of the list kernel
constexpr int kEwGroups = 16;        // energy/virial record groups (blocks b % 16; two per
                                      // XCD under the round-robin dispatch to 8 XCDs)
constexpr int kEwRecBytes = 128;     // one energy/virial record: 16 tagged 64-bit words
constexpr int kForceBlock = 256;
constexpr int kListBlock = 256;

}  // namespace relres

/*
 * relres.h -- C ABI of the MI355X (gfx950) Relative Resolution Lennard-Jones
 * hot path.
 *
 * The library evaluates the RelRes pair potential of Eq. 20 of "Relative
 * Resolution: A Computationally Efficient Implementation in LAMMPS"
 * (arXiv:2104.10231, Sec. 2.5) for a periodic orthorhombic box:
 *   - near atom pairs interact through the fine-grained (FG) LJ of Eq. 11,
 *     switched off between r_s- and r_s+ by the polynomial of Eqs. 16/17;
 *   - pairs of hybrid sites additionally interact through the coarse-grained
 *     (CG) LJ of Eq. 12, switched on over the same zone (Eq. 18) and off
 *     between r_c- and r_c+ (Eq. 17), shifted by the constants of Eq. 19;
 *   - ordinary sites carry no CG interaction (Eq. 14): a type is hybrid iff
 *     its CG energy parameter is positive (Sec. 2.5, correct use of lj/relres).
 * Instead of the single long-cutoff neighbour list of a conventional code it
 * builds the two lists described in Sec. 2.6: an atom list at r_s+ + skin over
 * all atoms and a site list at r_c+ + skin over hybrid atoms only.
 *
 * Conventions
 *   Units are the caller's (e.g. kcal/mol and Angstrom).  Positions are FP64,
 *   row-major N x 3, in caller order.  Forces come back in caller order.
 *   Energy is Eq. 3's total over non-excluded pairs; the virial is the pair
 *   virial tensor W_ab = sum_{i<j} (x_i - x_j)_a F_ij,b, with F_ij the force
 *   on i due to j, stored as {xx, yy, zz, xy, xz, yz}.
 *   "Device pointer" means memory from hipMalloc (or a torch CUDA/HIP tensor)
 *   on the current device.  The caller owns every pointer it passes; the
 *   library owns its context and all internal device buffers.
 *   `stream` is a hipStream_t (NULL = default stream).  All device work is
 *   enqueued on it; outputs are valid once the stream reaches that point.
 *   The context is not thread-safe; one context per device and host thread.
 *
 * Errors
 *   Every int-returning function returns RELRES_OK (0) or a negative
 *   RELRES_ERR_* code; relres_strerror() names it and relres_last_error()
 *   returns a message with details.  No C++ exception crosses the ABI.
 *   relres_build_lists and relres_check_lists may also return the positive
 *   RELRES_WARN_DANGEROUS_BUILD: the call succeeded (the lists are complete),
 *   but lists used before it had been kept too long.
 */
#ifndef RELRES_H
#define RELRES_H

#ifdef __cplusplus
extern "C" {
#endif

#define RELRES_ABI_VERSION 7

#define RELRES_OK                   0
#define RELRES_ERR_ARG             -1  /* null pointer, bad size or flag     */
#define RELRES_ERR_CUTOFF_ORDER    -2  /* r_s- <= r_s+ <= r_c- <= r_c+ and skin >= 0 violated */
#define RELRES_ERR_BOX_TOO_SMALL   -3  /* some L_k <= 2 (list radius)        */
#define RELRES_ERR_TOPOLOGY        -4  /* bad type / exclusion arrays        */
#define RELRES_ERR_HIP             -5  /* a HIP runtime call failed          */
#define RELRES_ERR_NO_LISTS        -6  /* forces requested before any build  */
#define RELRES_ERR_LIST_OVERFLOW   -7  /* list capacity could not be grown   */
#define RELRES_ERR_NONFINITE       -8  /* a position was NaN or infinite     */
#define RELRES_ERR_STATE           -9  /* call out of order                  */
#define RELRES_ERR_LIST_RETRY     -10  /* asynchronous build overflowed: rows grown, build again */
#define RELRES_ERR_STALE_LISTS    -11  /* dynamics: an atom moved more than half the skin between builds */
#define RELRES_ERR_EW_TIMEOUT     -12  /* a force call gave up waiting for its cross-block energy/virial
                                          sums (its energy and virial are NaN); see relres_sync */
/* Warning (positive; the call succeeded): this build found atoms more than
 * half the skin from where they were at the previous build of the same
 * topology and boxes, so forces computed from the previous lists may have
 * missed pairs (a "dangerous build" in Verlet-list terms).                 */
#define RELRES_WARN_DANGEROUS_BUILD  1

#define RELRES_MIX_GEOMETRIC   0   /* eps, sigma geometric means (Sec. 2.3)    */
#define RELRES_MIX_ARITHMETIC  1   /* Lorentz-Berthelot: eps geometric, sigma arithmetic */
#define RELRES_MIX_SIXTHPOWER  2   /* sigma_ab = ((sigma_a^6 + sigma_b^6)/2)^(1/6),
                                      eps_ab = 2 sqrt(eps_a eps_b) sigma_a^3 sigma_b^3
                                               / (sigma_a^6 + sigma_b^6)          */

#define RELRES_MAX_TYPES      32
#define RELRES_MAX_ATOMS      (1 << 27)
#define RELRES_MAX_EXCLUSIONS 64   /* excluded partners per atom, after symmetrisation */

/* Which neighbour list (relres_get_pairs). */
#define RELRES_LIST_ATOM  0   /* all non-excluded pairs, r < r_s+ + skin        */
#define RELRES_LIST_SITE  1   /* non-excluded hybrid pairs, r < r_c+ + skin     */

typedef struct relres_ctx relres_ctx;

/* Parameters of the pair style (Sec. 2.5: pair_style lj/relres r_s- r_s+ r_c-
 * r_c+, pair_coeff per type with optional distances, pair_modify shift and
 * mix).  Per-type arrays are host pointers of length ntypes, copied by
 * relres_create.  Mixed pair parameters are formed per type pair with `mix`,
 * for FG and CG alike.  An empty zone (r_- == r_+) is allowed (Sec. 2.5).
 * Distances: the global r_s-, r_s+, r_c-, r_c+ unless cut_type or cut_pair
 * is given.  With cut_type, type a keeps its own four distances and an
 * unlike pair mixes each distance with the sigma rule of `mix` (geometric
 * mixing gives the switching distance sqrt(r_s,a r_s,b) of Sec. 3.4); with
 * cut_pair every type pair has its own.  Every pair must satisfy r_s- <=
 * r_s+ <= r_c- <= r_c+; the atom list is then built at the largest r_s+ and
 * the site list at the largest r_c+ of a hybrid-hybrid pair (plus the skin).
 * The reference (conventional, all-FG) system of Sec. 2.1 is expressed as
 * r_s- = r_c(inner), r_s+ = r_c- = r_c+ = r_c(outer) with all eps_cg = 0.   */
typedef struct relres_params {
    double rs_in, rs_out, rc_in, rc_out;  /* r_s-, r_s+, r_c-, r_c+           */
    double skin;                          /* Verlet skin added to both lists  */
    int ntypes;                           /* 1 .. RELRES_MAX_TYPES            */
    const double *eps_fg, *sig_fg;        /* FG LJ per type (Eq. 11)          */
    const double *eps_cg, *sig_cg;        /* CG LJ per type (Eq. 12); eps_cg = 0 => ordinary */
    int mix;                              /* RELRES_MIX_*                     */
    int precision;                        /* force accumulation and output type:
                                             64 -> double* forces, 32 -> float* forces */
    int pair_math;                        /* type of the per-pair terms: 0 = same as
                                             precision, 32 or 64 (64 with precision 32
                                             evaluates pairs in FP64 and accumulates
                                             forces in FP32); energy and virial are
                                             always accumulated in FP64 */
    int no_shift;                         /* pair_modify shift: 0 = yes (Eq. 19, so
                                             u~(r_c+) = 0), 1 = no: Gamma_c- is zero
                                             where cases 3-4 of Eq. 20 subtract it,
                                             Gamma_s+- keep their Eq. 19 values (the
                                             energy then jumps by Gamma_c- at r_s+ and
                                             r_c+; forces are the same) */
    const double *cut_type;               /* NULL or ntypes x 4 {r_s-, r_s+, r_c-, r_c+} */
    const double *cut_pair;               /* NULL or ntypes x ntypes x 4, row-major
                                             [a][b][k], symmetric in a, b; takes
                                             precedence over cut_type */
} relres_params;

typedef struct relres_stats {
    long long n_atoms, n_sites;           /* atoms, hybrid atoms              */
    long long atom_entries, site_entries; /* full-list entries (each pair twice) */
    int atom_max_row, site_max_row;       /* longest row at the last build   */
    int atom_capacity, site_capacity;     /* allocated row capacity           */
    int atom_cells[3], site_cells[3];     /* cell grid of each list           */
    long long builds, regrows;            /* list builds, capacity regrows    */
    double box[3];                        /* box of the last build            */
    long long generation;                 /* changes whenever a device buffer that
                                             relres_forces reads or writes is
                                             reallocated; a graph that captured
                                             relres_forces must be re-captured then */
    long long dangerous_builds;           /* builds that returned (or, examined by
                                             another call, would have returned)
                                             RELRES_WARN_DANGEROUS_BUILD      */
    long long moved_at_last_build;        /* atoms the last examined build found
                                             more than half the skin from their
                                             previous-build positions          */
    int place_launches;                   /* launches that put the members of the
                                             last build into cell order: 1 (grids
                                             of at most 8192 cells, not crowded:
                                             per-cell buckets filled while binning,
                                             then one scan-and-sort launch) or 3
                                             (scan, scatter, cell sort); 0 before
                                             any build of a non-empty system    */
} relres_stats;

/* Create a context.  Validates the cutoff ordering r_s- <= r_s+ <= r_c- <=
 * r_c+ of every type pair (Sec. 2.5), mixes parameters and computes the
 * smoothing coefficients (Eqs. 17/18) and shifting constants (Eq. 19) in
 * FP64 on the host.  Binds the context to the current HIP device.  *out is
 * NULL on failure.                                                          */
int relres_create(const relres_params *params, relres_ctx **out);

/* CG parameters from FG ones, the parametrisation of Sec. 2.3 (host only, no
 * context or device needed).
 * Eq. 15, one CG site l made of n FG sites with per-site eps_fg[k],
 * sig_fg[k] (valid when the FG model mixes geometrically):
 *   B12 = sum_k sqrt(eps_k sig_k^12), B6 = sum_k sqrt(eps_k sig_k^6),
 *   sigma_l = (B12 / B6)^(1/3), eps_l = B6^4 / B12^2.
 * Eq. 13, one pair of CG sites from the n FG pair parameters eps_mn[k],
 * sig_mn[k] of all mu-nu pairs between them (any mixing):
 *   A12 = sum_k eps_k sig_k^12, A6 = sum_k eps_k sig_k^6,
 *   sigma_ij = (A12 / A6)^(1/6), eps_ij = A6^2 / A12.
 * n >= 1; eps >= 0 and sigma > 0 with a positive sum.  Results go to
 * *eps_cg, *sig_cg (host).                                                   */
int relres_cg_site_params(int n, const double *eps_fg, const double *sig_fg, double *eps_cg,
                          double *sig_cg);
int relres_cg_pair_params(int n, const double *eps_mn, const double *sig_mn, double *eps_cg,
                          double *sig_cg);

/* Mixed distance of two types under `mix` (the rule applied to cut_type for
 * unlike pairs): geometric sqrt(a b), arithmetic (a + b)/2, sixth-power
 * ((a^6 + b^6)/2)^(1/6).  Host only; returns NaN for an unknown rule.      */
double relres_mix_distance(int mix, double a, double b);

/* Atoms, by type and molecule (Sec. 3.1, data-file Atoms section), and the
 * pairs that do not interact at all (neither FG nor CG part): every pair of
 * one molecule if exclude_same_mol != 0, plus the CSR lists
 * excl_idx[excl_offsets[i] .. excl_offsets[i+1]) of caller indices (may be
 * NULL for none; they are symmetrised; at most RELRES_MAX_EXCLUSIONS partners
 * per atom).  Host arrays, copied.  types[i] must lie in [0, ntypes).
 * n_atoms may be 0.  Drops bonded terms and the dynamics setup, which refer
 * to the previous atoms.                                                     */
int relres_set_topology(relres_ctx *ctx, int n_atoms, const int *types, const int *mol,
                        int exclude_same_mol, const int *excl_offsets, const int *excl_idx);

/* Several independent systems (replicas) in one context: atoms
 * [atom_offsets[s], atom_offsets[s+1]) form system s (atom_offsets[0] = 0,
 * atom_offsets[nsys] = n_atoms, non-decreasing; host array, copied).  Each
 * system has its own periodic box and cell grids; pairs never cross
 * systems.  Every build, force and backward call then covers all systems in
 * one launch per step: boxes are nsys x 3, energies nsys x 3 and virials
 * nsys x 6.  relres_set_topology resets to one system.  With nsys > 1,
 * bonded terms and the dynamics setup are dropped.  Lists must be built
 * again afterwards.                                                         */
int relres_set_systems(relres_ctx *ctx, int nsys, const int *atom_offsets);

/* Skin of every system (host array of nsys values >= 0, Angstrom), in place
 * of relres_params.skin, from the next build on: each system's lists use
 * r_s+ + skin and r_c+ + skin, its box must exceed twice the larger, and its
 * displacement checks use half its skin.  Lets a batch keep the usual skin
 * where the boxes allow it and a smaller one in small boxes (a box edge must
 * exceed 2 (r_c+ + skin) for the minimum image to hold).  relres_set_topology
 * and relres_set_systems restore the default.  The lists must be built again
 * before relres_forces.                                                    */
int relres_set_skins(relres_ctx *ctx, const double *skins);

/* Build both neighbour lists for the FP64 device positions pos (N x 3, any
 * periodic image) in the box {Lx, Ly, Lz} (host array; nsys x 3 with
 * several systems).  Every L_k must exceed twice the largest list radius in
 * use (r_c+ + skin when the system has hybrid atoms, else r_s+ + skin).  Membership is decided in FP64 exactly as
 *   w = x - L floor(x/L), fixed into [0, L);
 *   d = w_j - w_i; d -= L if d > L/2; d += L if d < -L/2;
 *   r2 = (dx dx + dy dy) + dz dz;   member iff r2 < (r_+ + skin)^2
 * with separately rounded operations.  Synchronises `stream` once to check
 * the list capacity; grows the lists and rebuilds when a row overflowed.
 * Lists built with a skin stay exact while no atom has moved more than half
 * the skin since the build (the Verlet-list rule behind the paper's
 * neighbour lists, Sec. 2.6).  Each build checks this for the previous one
 * (same topology and boxes): RELRES_WARN_DANGEROUS_BUILD if some atom had
 * moved further; relres_moved_atoms checks it between builds.             */
int relres_build_lists(relres_ctx *ctx, const double *pos, const double box[3], void *stream);

/* The same build without waiting: everything is enqueued on `stream`, and
 * relres_forces may be enqueued behind it at once.  The lists are only known
 * to be complete once relres_check_lists has returned RELRES_OK; results
 * computed from them before that must be discarded if it does not.  The first
 * build of a context, and any build after the cell grid or the capacities
 * changed, waits as relres_build_lists does.  A status left unexamined is
 * examined by the next build, relres_list_stats or relres_get_pairs (which
 * then report its non-finite-position error).                              */
int relres_build_lists_async(relres_ctx *ctx, const double *pos, const double box[3],
                             void *stream);
/* A build enqueued on a stream that is being captured into a HIP graph runs
 * at every replay of the graph.  Its status accumulates on the device, and
 * relres_check_lists copies it to the host itself and examines every replay
 * since the previous check at once (one check after many replays is enough):
 * synchronise the stream after the replays first.  RELRES_ERR_LIST_RETRY
 * there (some replay overflowed a row) grows the rows, which changes the
 * buffer generation (relres_generation): capture again and redo the
 * replays.  Timing events are not recorded during capture.                */

/* Waits for the status of the last build and examines it: RELRES_OK when the
 * lists are complete, RELRES_ERR_NONFINITE for a NaN/inf position, or
 * RELRES_ERR_LIST_RETRY when a row overflowed its capacity: the capacity has
 * been grown and the lists are invalid until the next build.  Waits only for
 * the build itself, not for work enqueued after it.  Complete lists from a
 * build that found atoms past half the skin (see relres_build_lists) give
 * RELRES_WARN_DANGEROUS_BUILD instead of RELRES_OK, once per such build.   */
int relres_check_lists(relres_ctx *ctx);

/* Waits for all work on `stream` and reports what force calls since the
 * previous report left in the device status: RELRES_ERR_EW_TIMEOUT if the
 * cross-block energy/virial reduction of some call (one system) gave up
 * waiting for other blocks (a bounded wait; that call's energy and virial are
 * NaN, its forces are valid).  relres_check_lists reports it too for calls
 * enqueued before the build it examines.  Not allowed while `stream` is
 * being captured (RELRES_ERR_STATE).                                       */
int relres_sync(relres_ctx *ctx, void *stream);

/* Number of atoms of pos (device, N x 3 FP64) that are more than half the
 * skin (minimum image, the box of their system) from where they were at the
 * last build; 0 means the lists are still exact for pos (Sec. 2.6 Verlet
 * lists: rebuild when it is not, e.g. every few steps as LAMMPS's "check
 * yes" does).  A non-finite position counts as moved.  Enqueues one small
 * kernel on `stream` and waits for it (not allowed while the stream is being
 * captured: RELRES_ERR_STATE).  RELRES_ERR_NO_LISTS before the first build.
 * count: host int.                                                          */
int relres_moved_atoms(relres_ctx *ctx, const double *pos, void *stream, int *count);

/* Forces, energy and virial for device positions pos (N x 3 FP64) using the
 * lists of the last build (and its box).  forces: device N x 3, double* when
 * precision == 64, float* when 32; overwritten.  energy: device double[3] =
 * {total, FG part, CG part} or NULL; virial: device double[6] or NULL (per
 * system, nsys x 3 and nsys x 6, with several systems).
 * Energy and virial are accumulated in FP64 and reduced in a fixed order, so
 * repeated calls are bitwise identical.  Asynchronous on `stream`.          */
int relres_forces(relres_ctx *ctx, const double *pos, void *forces, double *energy,
                  double *virial, void *stream);

/* relres_forces for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * The same kernels and results, bit for bit; the energy/virial scratch
 * (launch epoch and per-block records) lives in a static device array of
 * RELRES_NOALLOC_SCRATCH_BYTES that the library holds on each GPU until the
 * process ends, instead of context buffers.  Nothing is allocated or freed:
 * the caller passes the outputs, and the lists come from the last
 * relres_build_lists.  RELRES_ERR_ARG when the launch would need more scratch
 * than the array holds (256 bytes, then 128 for every block of 256 threads
 * and for each of 16 record groups: up to 16366 blocks, e.g. a million rows
 * at 4 lanes per row) or, with energy or virial requested, for several
 * systems (their per-row partials need context buffers; forces only is
 * fine).  Every call on one GPU shares that GPU's array: calls that overlap
 * on one GPU (several streams, threads or contexts at once) race and must be
 * serialised by the caller.  No timing events are recorded.  Asynchronous on
 * `stream`.                                                               */
#define RELRES_NOALLOC_SCRATCH_BYTES (2 << 20)
int relres_forces_noalloc(relres_ctx *ctx, const double *pos, void *forces, double *energy,
                          double *virial, void *stream);

/* Replace the pair parameters (Sec. 2.3 mixing bypassed): host arrays of
 * ntypes*ntypes doubles, row-major [a][b] (ordered entries; a symmetric
 * table describes the usual physics).  The FG entries need eps >= 0 and
 * sigma > 0; the CG entries are used only for hybrid-hybrid type pairs
 * (where they need eps >= 0, sigma > 0) and are zero otherwise (Eq. 14).
 * Recomputes every coefficient of Eqs. 17-19 on the host and uploads them;
 * waits for the device first.  Lists stay valid.                          */
int relres_set_pair_params(relres_ctx *ctx, const double *eps_fg, const double *sig_fg,
                           const double *eps_cg, const double *sig_cg);

/* Adjoint of relres_forces for J = e_bar * E + sum_i g_i . F_i, where E is
 * the total energy (Eq. 3) and F the forces, at the device positions pos
 * (N x 3 FP64) with the lists of the last build:
 *   grad_forces  device N x 3 FP64: g = dJ/dF (NULL: zero);
 *   grad_energy  device double[nsys]: e_bar = dJ/dE of each system's
 *                total energy (NULL: zero);
 *   grad_pos     device N x 3 FP64, overwritten with dJ/dx;
 *   grad_pair    device double[4 * ntypes * ntypes], overwritten with dJ/dP
 *                for P = eps_FG, sigma_FG, eps_CG, sigma_CG (that order),
 *                each [a][b] row-major, treating the ordered pair entries
 *                as independent (relres_backward_types carries them through
 *                the mixing rule to the per-type values).
 * Pair terms are recomputed (FP64), nothing is stored by relres_forces.
 * Parameter sums are reduced in a fixed order (bitwise repeatable).  At most
 * 8 types: the kernel bins its parameter sums per neighbour type in
 * registers (8 x 4 FP64 per lane), and more bins would cut its occupancy;
 * RELRES_ERR_ARG beyond.  Asynchronous on `stream`.                        */
int relres_backward(relres_ctx *ctx, const double *pos, const double *grad_forces,
                    const double *grad_energy, double *grad_pos, double *grad_pair,
                    void *stream);

/* Replace the per-type parameters (host arrays of ntypes doubles each, as in
 * relres_params) and mix them again with the context's rule (Sec. 2.3; CG
 * pair parameters only for hybrid-hybrid pairs, Eq. 14).  The hybrid types
 * are fixed by relres_create (they define the site list): a hybrid type keeps
 * eps_cg > 0 and sigma_cg > 0, an ordinary one eps_cg = 0, else
 * RELRES_ERR_ARG.  Recomputes every coefficient of Eqs. 17-19 on the host and
 * uploads them; waits for the device first.  Lists stay valid.             */
int relres_set_type_params(relres_ctx *ctx, const double *eps_fg, const double *sig_fg,
                           const double *eps_cg, const double *sig_cg);

/* relres_backward with the parameter gradient carried through the mixing
 * rule of Sec. 2.3 to the per-type values of relres_create or the last
 * relres_set_type_params:
 *   grad_type  device double[4 * ntypes], overwritten with dJ/d eps_FG,
 *              dJ/d sigma_FG, dJ/d eps_CG, dJ/d sigma_CG of each type (that
 *              order, ntypes values each).  The CG values of ordinary types
 *              get 0: Eq. 14 fixes their pair parameters at zero.
 * The other arguments are those of relres_backward.  The per-type values
 * must be positive (FG of every type, CG of hybrid types): the mixing rules
 * have no derivative at zero (RELRES_ERR_ARG).  RELRES_ERR_STATE after
 * relres_set_pair_params, whose tables have no per-type values.  Uses a
 * library-owned buffer for the pair gradients: calls on one context must not
 * overlap.  Asynchronous on `stream`.                                       */
int relres_backward_types(relres_ctx *ctx, const double *pos, const double *grad_forces,
                          const double *grad_energy, double *grad_pos, double *grad_type,
                          void *stream);

/* Bonded terms and scaled 1-4 pairs of the molecular model (Sec. 3.2: AMBER
 * united-atom bonds, angles and Fourier dihedrals, 1-4 non-bonded pairs
 * scaled down by a factor 2).  Host arrays, copied; atom indices in caller
 * order, in [0, n_atoms) of the topology:
 *   bonds     nbonds x 2 (i, j);         E = bond_k (r - bond_r0)^2
 *   angles    nangles x 3 (i, j, k), j the vertex;
 *                                        E = angle_k (theta - angle_t0)^2
 *   dihedrals ndihedrals x 4 (i, j, k, l);
 *                                        E = dih_k (1 + cos(dih_n phi - dih_d)),
 *             phi the IUPAC dihedral (trans = pi)
 *   pairs14   npairs14 x 2: these pairs interact through the pair potential
 *             of Eq. 20 (FG and CG parts, their own distances) times
 *             scale14; they should be excluded from the lists
 *             (relres_set_topology) so that they are not counted twice.
 * Spring constants follow the AMBER convention (no factor 1/2).  Requires a
 * single system; replaces any earlier set; waits for the device first.     */
int relres_set_bonded(relres_ctx *ctx, int nbonds, const int *bonds, const double *bond_k,
                      const double *bond_r0, int nangles, const int *angles,
                      const double *angle_k, const double *angle_t0, int ndihedrals,
                      const int *dihedrals, const double *dih_k, const int *dih_n,
                      const double *dih_d, int npairs14, const int *pairs14, double scale14);

/* Bonded and scaled 1-4 forces at the device positions pos (N x 3 FP64),
 * ADDED to forces (device, the type of relres_forces), with the box of the
 * last build.  energy: device double[4] = {bonds, angles, dihedrals, 1-4
 * pairs} or NULL; virial: device double[6] (their pair/term virial, the
 * convention of relres_forces) or NULL.  FP64 throughout; every atom sums
 * the terms it belongs to in a fixed order (deterministic, no atomics).
 * Asynchronous on `stream`.                                                */
int relres_bonded_forces(relres_ctx *ctx, const double *pos, void *forces, double *energy,
                         double *virial, void *stream);

/* Dynamics in the canonical ensemble (Sec. 3.2): velocity Verlet with one
 * Nose-Hoover thermostat, propagated in symmetric half steps
 *   xi += dt/4 G; v *= exp(-xi dt/2); eta += dt/2 xi; xi += dt/4 G,
 *   G = (2K - g kT)/Q, g = 3N - 3, Q = g kT tau^2,
 * around v += dt/2 a; x += dt v; forces; v += dt/2 a.
 * masses: host double[n] (caller order); dt, tau: time unit of the caller;
 * kT: energy unit; ftm2v converts force / mass to acceleration (4.184e-4 for
 * kcal/mol, A, amu and fs).  The lists are rebuilt every rebuild_every steps
 * (waiting for each build); if an atom moved more than half the skin since
 * the previous build, relres_md_run fails with RELRES_ERR_STALE_LISTS.
 * Resets the thermostat to xi = eta = 0.                                   */
int relres_md_setup(relres_ctx *ctx, const double *masses, double dt, double kT, double tau,
                    double ftm2v, int rebuild_every);

/* Read (set = 0) or write (set = 1) the thermostat state xi, eta (host
 * doubles).  Waits for the device.                                        */
int relres_md_state(relres_ctx *ctx, double *xi, double *eta, int set);

/* Run nsteps steps from the device positions pos and velocities vel (N x 3
 * FP64 each, updated in place; positions are never wrapped), in the box of
 * the last build.  Forces come from relres_forces (the context's precision)
 * plus relres_bonded_forces when bonded terms are set.  With thermo_every >
 * 0, every thermo_every-th step appends one row of 8 doubles to the device
 * buffer thermo (nsteps / thermo_every rows): non-bonded energy (Eq. 3), 1-4
 * energy, bond, angle and dihedral energies, kinetic energy, the extended
 * energy K + U + Q xi^2/2 + g kT eta (conserved by the integrator), and the
 * trace of the virial.  Enqueued on `stream`; waits at every list build and
 * at the end.                                                              */
int relres_md_run(relres_ctx *ctx, double *pos, double *vel, int nsteps, int thermo_every,
                  double *thermo, void *stream);

/* List statistics of the last build (host struct).  Entry counts and row
 * lengths are computed on demand by a small kernel the first time they are
 * asked for after a build, which synchronises the device.                   */
int relres_list_stats(relres_ctx *ctx, relres_stats *out);

/* Cheap query (no device work): the buffer generation of relres_stats.  A
 * HIP graph that captured relres_forces stays valid while it is unchanged.  */
int relres_generation(relres_ctx *ctx, long long *generation);

/* Copy one list as canonical caller-index pairs (i, j), i < j, sorted by i
 * then j, into pairs_host (2*cap ints).  *n_out receives the number of pairs,
 * which may exceed cap (then only cap are written).  Synchronises.         */
int relres_get_pairs(relres_ctx *ctx, int which, int *pairs_host, long long cap,
                     long long *n_out);

/* Lanes of a wavefront that share one list row in the force kernel: for rows
 * of ordinary atoms (atom list) and of hybrid atoms (atom + site list).
 * Powers of two up to 64; 0 selects a value from the mean row length of the
 * last build (about 4 entries per lane, 8 or 16 in launches that fill the
 * GPU many times over).                                                    */
int relres_set_launch(relres_ctx *ctx, int lanes_atom, int lanes_site);

/* Shape of the list-build kernel: home rows per wavefront for the atom grid
 * and for the site grid (1..16, 0 = automatic: 8, or 16 in launches of many
 * waves, fewer in small launches) and candidates held per lane (2 or 4, 0 =
 * automatic: 4 when every wave of the launch is resident at once).  Takes
 * effect at the next build; the lists themselves (pairs and their order in a
 * row) do not depend on it.  Overrides persist until changed.               */
int relres_set_list_launch(relres_ctx *ctx, int rows_atom, int rows_site, int cand_per_lane);

/* Cell size of the list grids (Sec. 2.6 cell lists): cells per list radius
 * along an axis for the atom grid and for the site grid, 1 (cells of at least
 * the list radius, a 27-cell stencil) or 2 (cells of at least half of it, a
 * 125-cell stencil: about 42 % less volume to search per row, more cells and
 * fewer rows sharing a stencil), 0 = automatic (1).  Takes effect at the next
 * build; the pair sets do not depend on it (the order of a row's entries
 * does).  Overrides persist until changed.                                 */
int relres_set_cells(relres_ctx *ctx, int div_atom, int div_site);

/* Result of relres_autotune (host struct).  Chosen shapes (resolved, never
 * 0), mean device times of the chosen and of the automatic shapes, and the
 * number of shapes timed.                                                   */
typedef struct relres_tune {
    int rows_atom, rows_site, cand_per_lane;   /* list kernel                 */
    int lanes_atom, lanes_site;                /* force kernel                */
    int trials;
    double build_us, build_us_auto;            /* one list build              */
    double force_us, force_us_auto;            /* one force call with E and W */
    int cell_div_atom, cell_div_site;          /* cells per list radius       */
} relres_tune;

/* Autotuner for the caller's own workload: times list builds for every cell
 * size of each grid (relres_set_cells 1 or 2) and list kernel shape (rows per
 * wave 4/8/16 for each grid x 2/4 candidates per lane), and the automatic
 * choice, on the device positions pos and box(es),
 * keeps the fastest, rebuilds, then times force calls (with energy and
 * virial) for lanes per row 2..16 (atom rows) x 2..32 (hybrid rows) and the
 * automatic choice, and keeps the fastest.  Each shape: one untimed call,
 * then reps (1..1000) timed with HIP events on `stream`.  Leaves valid lists
 * built from pos and the chosen shapes set (as by relres_set_cells,
 * relres_set_list_launch and relres_set_launch).  Synchronises; allocates temporary force, energy and
 * virial buffers; must not run on a capturing stream (RELRES_ERR_STATE).
 * Resets the relres_get_timing tallies.  Writes *out.  On an error the
 * shapes set before the call are restored; build the lists again before the
 * next force call.                                                          */
int relres_autotune(relres_ctx *ctx, const double *pos, const double *box, void *stream, int reps,
                    relres_tune *out);

/* With enable != 0, HIP events are recorded on the caller's stream right
 * before and after every launch of the force kernel (which includes the
 * energy/virial reduction) and around every list build.
 * relres_get_timing synchronises, returns the accumulated milliseconds and
 * launch counts since the previous call, and resets them.                  */
int relres_set_timing(relres_ctx *ctx, int enable);
int relres_get_timing(relres_ctx *ctx, double *force_ms, long long *force_calls,
                      double *build_ms, long long *build_calls);

/* Free the context and all of its device memory (NULL is allowed). */
void relres_destroy(relres_ctx *ctx);

const char *relres_strerror(int code);
/* Detail of the most recent error on this thread (never NULL). */
const char *relres_last_error(void);
int relres_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RELRES_H */

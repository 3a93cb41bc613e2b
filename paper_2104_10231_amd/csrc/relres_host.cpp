// relres_host.cpp -- C ABI of the RelRes Lennard-Jones hot path: parameter
// setup in FP64 on the host, device memory management, and the call sequences
// of relres_build_lists and relres_forces (kernels in relres_kernels.hip).
#include "relres.h"
#include "relres_internal.h"

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

using namespace relres;

namespace {

thread_local std::string g_last_error = "no error";

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t _e = (expr);                                                             \
        if (_e != hipSuccess)                                                               \
            return fail(RELRES_ERR_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), \
                        __FILE__, __LINE__);                                                \
    } while (0)

#define TRY(expr)                  \
    do {                           \
        int _rc = (expr);          \
        if (_rc != RELRES_OK) return _rc; \
    } while (0)

// ---------------------------------------------------------------------------
// FP64 parameter setup (Secs. 2.3-2.5)
// ---------------------------------------------------------------------------

struct LJ3 {
    double u, du, d2u;   // u, du/dr, d2u/dr2 of Eq. 11 / Eq. 12
};

LJ3 lj3(double eps, double sig, double r)
{
    const double q2 = (sig / r) * (sig / r);
    const double q6 = q2 * q2 * q2;
    const double q12 = q6 * q6;
    return {4.0 * eps * (q12 - q6), 24.0 * eps / r * (q6 - 2.0 * q12),
            24.0 * eps / (r * r) * (26.0 * q12 - 7.0 * q6)};
}

// Eq. 17: polynomial that switches a potential off over [r_-, r_- + D),
// matching u, u', u'' at r_- and with vanishing f', f'' at the far end (Eq. 7).
// An empty zone keeps only the constant term.
void switch_off(const LJ3& u, double D, double g[5])
{
    g[0] = u.u;
    if (D == 0.0) {
        g[1] = g[2] = g[3] = g[4] = 0.0;
        return;
    }
    g[1] = u.du;
    g[2] = 0.5 * u.d2u;
    g[3] = -u.du / (D * D) - 2.0 * u.d2u / (3.0 * D);
    g[4] = u.du / (2.0 * D * D * D) + u.d2u / (4.0 * D * D);
}

// Eq. 18: polynomial that switches a potential on over [r_+ - D, r_+) with
// f', f'' vanishing at the near end and matching u, u', u'' at r_+ (Eq. 8).
// gamma_4+ carries +u''/(4 D^2): with the sign printed in Eq. 18 the second
// derivative at r_+ would be -5 u'' instead of u''.
void switch_on(const LJ3& u, double D, double g[5])
{
    g[1] = g[2] = 0.0;
    if (D == 0.0) {
        g[0] = u.u;
        g[3] = g[4] = 0.0;
        return;
    }
    g[0] = u.u - 0.5 * u.du * D + u.d2u * D * D / 12.0;
    g[3] = u.du / (D * D) - u.d2u / (3.0 * D);
    g[4] = -u.du / (2.0 * D * D * D) + u.d2u / (4.0 * D * D);
}

double poly_at(const double g[5], double d)
{
    return g[0] + d * (g[1] + d * (g[2] + d * (g[3] + d * g[4])));
}

// Mixed length (sigma, or a distance of per-type cutoffs) of two types.
double mix_sigma(int mix, double a, double b)
{
    if (mix == RELRES_MIX_ARITHMETIC) return 0.5 * (a + b);
    if (mix == RELRES_MIX_SIXTHPOWER) {
        const double a3 = a * a * a, b3 = b * b * b;
        return std::pow(0.5 * (a3 * a3 + b3 * b3), 1.0 / 6.0);
    }
    return std::sqrt(a * b);
}

// Mixed energy of two types; the sixth-power rule keeps eps sigma^6 a
// geometric mean, so it depends on the sigmas too.
double mix_eps(int mix, double ea, double eb, double sa, double sb)
{
    if (mix == RELRES_MIX_SIXTHPOWER) {
        const double a3 = sa * sa * sa, b3 = sb * sb * sb;
        return 2.0 * std::sqrt(ea * eb) * a3 * b3 / (a3 * a3 + b3 * b3);
    }
    return std::sqrt(ea * eb);
}

// Derivatives of a mixed pair (eps_ab, sigma_ab) with respect to the values
// of type a (the first argument), from the definitions of the rules:
//   geometric        eps_ab = sqrt(ea eb), sigma_ab = sqrt(sa sb)
//   Lorentz-Berthelot  eps_ab as geometric, sigma_ab = (sa + sb) / 2
//   sixth-power      eps_ab = 2 sqrt(ea eb) sa^3 sb^3 / (sa^6 + sb^6),
//                    sigma_ab = ((sa^6 + sb^6) / 2)^(1/6)
// out = {d eps_ab/d ea, d eps_ab/d sa, d sigma_ab/d sa} (sigma_ab does not
// depend on the energies).  Type b's derivatives follow by swapping the
// arguments.  The values must be positive.
void mix_derivs(int mix, double ea, double eb, double sa, double sb, double out[3])
{
    const double e = mix_eps(mix, ea, eb, sa, sb);
    out[0] = 0.5 * e / ea;
    if (mix == RELRES_MIX_SIXTHPOWER) {
        const double a3 = sa * sa * sa, b3 = sb * sb * sb;
        const double s6 = a3 * a3 + b3 * b3;
        const double s = mix_sigma(mix, sa, sb);
        out[1] = e * (3.0 / sa - 6.0 * a3 * sa * sa / s6);
        out[2] = a3 * sa * sa / (2.0 * s * s * s * s * s);
        return;
    }
    out[1] = 0.0;
    out[2] = mix == RELRES_MIX_ARITHMETIC ? 0.5 : 0.5 * std::sqrt(sb / sa);
}

// u, u', u'' (wrt = 0) or their derivatives with respect to eps (wrt = 1) or
// sigma (wrt = 2).  u is linear in eps; with q = sigma/r the sigma
// derivatives are 4 eps (12 q^12 - 6 q^6)/sigma, 24 eps (6 q^6 - 24 q^12)/(r
// sigma) and 24 eps (312 q^12 - 42 q^6)/(r^2 sigma).
LJ3 lj3_wrt(double eps, double sig, double r, int wrt)
{
    if (wrt == 0) return lj3(eps, sig, r);
    if (wrt == 1) return lj3(1.0, sig, r);
    const double q2 = (sig / r) * (sig / r);
    const double q6 = q2 * q2 * q2;
    const double q12 = q6 * q6;
    return {4.0 * eps * (12.0 * q12 - 6.0 * q6) / sig, 24.0 * eps / (r * sig) * (6.0 * q6 - 24.0 * q12),
            24.0 * eps / (r * r * sig) * (312.0 * q12 - 42.0 * q6)};
}

// A eps sigma^n, or its derivative with respect to eps (wrt 1) or sigma (wrt 2)
double power_term(double A, double eps, double sig, int n, int wrt)
{
    double p = 1.0;
    for (int k = 0; k < (wrt == 2 ? n - 1 : n); ++k) p *= sig;
    return wrt == 0 ? A * eps * p : wrt == 1 ? A * p : n * A * eps * p;
}

// FG part of a pair record (LJ constants of Eq. 11, f_s-^FG of Eq. 17 and its
// end value), or its derivative with respect to eps / sigma.  Every field is
// linear in (A eps sigma^n) terms and in u, u', u'' at r_s- (Eqs. 17, 19), so
// differentiating the inputs differentiates the record.
void fg_part(PairCoef<double>& k, double e, double s, int wrt, double rsi, double Ds)
{
    k.fg_c12 = power_term(48.0, e, s, 12, wrt);
    k.fg_c6 = power_term(24.0, e, s, 6, wrt);
    k.fg_e12 = power_term(4.0, e, s, 12, wrt);
    k.fg_e6 = power_term(4.0, e, s, 6, wrt);
    switch_off(lj3_wrt(e, s, rsi, wrt), Ds, k.fg_g);
    k.fg_shift = poly_at(k.fg_g, Ds);
}

// CG part: LJ constants of Eq. 12, f_s+^CG (Eq. 18), f_c-^CG (Eq. 17) and
// Gamma_c- (Eq. 19), or their derivatives.  Cases 1-2 of Eq. 20 always carry
// Gamma_c- (inside Gamma_s+-); cases 3-4 carry it unless no_shift.
void cg_part(PairCoef<double>& k, double e, double s, int wrt, double rso, double rci, double Ds,
             double Dc, int no_shift)
{
    k.cg_c12 = power_term(48.0, e, s, 12, wrt);
    k.cg_c6 = power_term(24.0, e, s, 6, wrt);
    k.cg_e12 = power_term(4.0, e, s, 12, wrt);
    k.cg_e6 = power_term(4.0, e, s, 6, wrt);
    double g[5];
    switch_on(lj3_wrt(e, s, rso, wrt), Ds, g);
    k.sp_g0 = g[0];
    k.sp_g3 = g[3];
    k.sp_g4 = g[4];
    switch_off(lj3_wrt(e, s, rci, wrt), Dc, k.cm_g);
    k.sp_shift = poly_at(k.cm_g, Dc);
    k.cm_shift = no_shift ? 0.0 : k.sp_shift;
}

// Distances of one type pair with their squares.
template <typename S>
Cutoffs<S> cutoffs_of(const double* r4)
{
    Cutoffs<S> c;
    c.rsi = (S)r4[0]; c.rso = (S)r4[1]; c.rci = (S)r4[2]; c.rco = (S)r4[3];
    c.rsi2 = (S)(r4[0] * r4[0]); c.rso2 = (S)(r4[1] * r4[1]);
    c.rci2 = (S)(r4[2] * r4[2]); c.rco2 = (S)(r4[3] * r4[3]);
    return c;
}

// ---------------------------------------------------------------------------
// device memory
// ---------------------------------------------------------------------------

struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    template <typename T> T* as() const { return static_cast<T*>(p); }
};

// Grow a device buffer.  `gen` counts (re)allocations of the buffers of one
// context: device pointers that a graph captured are stale once it changes.
int ensure(DBuf& b, size_t bytes, long long* gen)
{
    if (bytes == 0) bytes = 64;
    if (b.p && b.bytes >= bytes) return RELRES_OK;
    ++*gen;
    if (b.p) HIP_TRY(hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
    HIP_TRY(hipMalloc(&b.p, bytes));
    b.bytes = bytes;
    return RELRES_OK;
}

void release(DBuf& b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

// All cell grids of one kind (atom or site), one per system, concatenated.
struct GridHost {
    double rl = 0.0;
    int cap = 0;
    int nsys = 0;
    int ncell = 0;                    // cells of all grids
    int members = 0;                  // members of all grids
    int waves = 0;                    // list-kernel waves (rpw rows each)
    int rpw = 8;                      // home rows per list-kernel wave
    int div = 1;                      // cells per list radius along an axis: 1 (27-cell
                                      // stencil) or 2 (cells of half the radius, 125 cells)
    bool site = false;                // the site grid (hybrid atoms)
    int n[3] = {0, 0, 0};             // cells per axis of system 0 (statistics)
    std::vector<int> sys_n;           // [nsys][3] cells per axis
    std::vector<GeomDev> geom;        // per system, as last uploaded
    std::vector<int> wave_sys;        // system of every list-kernel wave, as last uploaded
    DBuf geom_dev, wave_sys_dev, cell_sys, rank_of_lin, lin_of_rank, nbr, count, start, user_unsorted, user, pos,
        meta, row_cell, list, nrow;
    GridDev dev{};
};

uint32_t spread3(uint32_t v)
{
    uint32_t r = 0;
    for (int b = 0; b < 10; ++b) r |= ((v >> b) & 1u) << (3 * b);
    return r;
}

}  // namespace

struct relres_ctx {
    int device = 0;
    double skin = 0;                  // default skin of every system
    std::vector<double> skins;        // per system (relres_set_skins); empty: `skin`
    std::vector<double> ref_skins;    // skins of the build whose positions wpos holds
    std::vector<double> dist;         // [pair][4]: r_s-, r_s+, r_c-, r_c+ of each type pair
    bool per_pair = false;            // distances differ between type pairs
    double list_rso = 0, list_rco = 0;   // largest r_s+; largest hybrid-pair r_c+
    int ntypes = 0, mix = 0, precision = 64, pair_math = 64, no_shift = 0;
    std::vector<int> hybrid;
    std::vector<PairCoef<double>> coef64;     // per type pair
    std::vector<PairCoef<double>> coef_grad;  // [4][pair]: d/d eps_FG, sigma_FG, eps_CG, sigma_CG
    // per-type parameters the pair tables were mixed from (relres_create,
    // relres_set_type_params); false after relres_set_pair_params, which
    // bypasses the mixing (per-type gradients are then undefined)
    std::vector<double> type_par;     // [4][ntypes]: eps_FG, sigma_FG, eps_CG, sigma_CG
    bool tables_from_types = true;
    DBuf d_mix_jac, d_gpair;          // mixing Jacobian (see mix_jacobian); pair gradients
    DBuf d_coef64, d_coef32, d_hybrid, d_coef_grad, d_bpartial, d_pcut64, d_pcut32;
    double cut64[8] = {0};            // the distances of every pair when !per_pair

    bool topo_set = false;
    int n = 0, n_sites = 0;
    int nsys = 1;                     // systems (atoms grouped by system)
    std::vector<int> sys_off;         // [nsys + 1] first atom of each system
    std::vector<int> atoms_sys, sites_sys;   // atoms and hybrid atoms per system
    std::vector<int> h_types;         // types of the atoms (host copy)
    DBuf d_sys;                       // system of each atom (nsys > 1)
    std::vector<double> boxes;        // [nsys][3] of the last build
    std::vector<double> boxes_dev;    // [nsys][6] as uploaded
    DBuf d_boxes, d_row_ew, d_wave_ew, d_wave_sys;
    int same_mol = 0;
    bool has_excl = false;
    int max_excl = 0;
    DBuf d_types, d_mol, d_excl_off, d_excl_idx;

    GridHost ga, gs;
    DBuf d_grids, d_wpos, d_key_a, d_key_s, d_user2arow, d_a_rec, d_s_rec, d_status, d_seg_tot;
    GridDev* h_grids = nullptr;       // pinned staging of the device descriptors
    GridDev uploaded[2] = {};         // descriptors currently on the device
    bool grids_valid = false;
    Status* h_status = nullptr;
    Status* h_query = nullptr;        // pinned landing place of relres_moved_atoms
    int nonfinite_seen = 0;
    unsigned moved_seen = 0;          // Status::moved at the last examination
    unsigned ew_failed_seen = 0;      // Status::ew_failed at the last examination
    int spin_limit = 1 << 22;         // polls before a cross-block energy/virial wait gives up
    bool place_one_launch = true;     // grids of few cells: scan, scatter and sort in one launch
    bool ref_valid = false;           // wpos holds a previous build of this topology
    bool warn_pending = false;        // a build found atoms past half the skin, not yet reported
    bool stats_fresh = false;         // statistics describe the current lists
    bool lanes_stale = true;          // automatic lane counts need a refresh
    bool built = false;
    bool check_pending = false;       // a build's status has not been examined yet
    bool status_in_graph = false;     // ... and it was captured into a graph: no event
    hipEvent_t ev_status = nullptr;   // recorded after a build's status copy
    hipEvent_t ev_upload = nullptr;   // recorded after the descriptor upload
    bool upload_pending = false;
    double box[3] = {0, 0, 0};

    DBuf d_partials, d_epoch;
    void* scratch = nullptr;          // this device's static scratch (relres_forces_noalloc)
    hipError_t scratch_err = hipSuccess;
    int lanes_a = 0, lanes_b = 0;        // caller override, 0 = automatic
    int auto_la = 4, auto_lb = 16;
    // list kernel shape: rows per wave (atom, site grids) and candidates per
    // lane; caller or autotuner override, 0 = automatic
    int rows_a = 0, rows_s = 0, cand = 0;
    // cells per list radius of the atom and the site grid (relres_set_cells
    // or the autotuner; 0 = automatic, which is 1)
    int div_a = 0, div_s = 0;

    relres_stats stats{};
    long long alloc_generation = 0;

    // bonded terms and scaled 1-4 pairs (relres_set_bonded)
    bool has_bonded = false;
    double scale14 = 0.0;
    DBuf d_items, d_bond_par, d_angle_par, d_dih_par, d_bond_part, d_bond_sum;
    int bond_slots = 1;               // bonded items per atom (padded)
    int bond_lg = 0;                  // lanes per atom of the bonded kernel = 2^bond_lg
    // dynamics (relres_md_setup / relres_md_run)
    bool md_ready = false;
    double md_ftm2v = 0.0;
    int md_rebuild = 10;
    int md_cur = 0;                   // which of the two state buffers is current
    DBuf d_mass, d_md_state, d_md_xref, d_md_F, d_md_E, d_md_W, d_md_part, d_md_stale;
    unsigned int* h_stale = nullptr;

    bool timing = false;
    std::vector<hipEvent_t> ev_free;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_force, ev_build;
    double force_ms = 0, build_ms = 0;
    long long force_calls = 0, build_calls = 0;
};

namespace {

// Coefficient records of every type pair from pair tables (row-major
// [a][b]): the record of Eq. 20's FG and CG parts, and its derivatives with
// respect to the four pair parameters.  The CG part of a pair that is not
// hybrid-hybrid is zero (Eq. 14).
void build_tables(relres_ctx* c, const double* ef, const double* sf, const double* ec,
                  const double* sc)
{
    const int nt = c->ntypes;
    const size_t np = (size_t)nt * nt;
    c->coef64.assign(np, PairCoef<double>{});
    c->coef_grad.assign(4 * np, PairCoef<double>{});
    const int ns = c->no_shift;
    for (int a = 0; a < nt; ++a)
        for (int b = 0; b < nt; ++b) {
            const size_t q = (size_t)a * nt + b;
            const double* r = &c->dist[4 * q];
            const double Ds = r[1] - r[0], Dc = r[3] - r[2];
            fg_part(c->coef64[q], ef[q], sf[q], 0, r[0], Ds);
            fg_part(c->coef_grad[0 * np + q], ef[q], sf[q], 1, r[0], Ds);
            fg_part(c->coef_grad[1 * np + q], ef[q], sf[q], 2, r[0], Ds);
            if (c->hybrid[a] && c->hybrid[b]) {
                cg_part(c->coef64[q], ec[q], sc[q], 0, r[1], r[2], Ds, Dc, ns);
                cg_part(c->coef_grad[2 * np + q], ec[q], sc[q], 1, r[1], r[2], Ds, Dc, ns);
                cg_part(c->coef_grad[3 * np + q], ec[q], sc[q], 2, r[1], r[2], Ds, Dc, ns);
            }
        }
}

// Pair tables mixed from per-type parameters (Sec. 2.3 with the context's
// `mix` rule; CG pair parameters only for hybrid-hybrid pairs, Eq. 14), the
// coefficient records built from them, and the mixing Jacobian that carries
// pair gradients back to the per-type values (relres_backward_types):
// [family FG/CG][pair q = a*nt + b][6] = d eps_ab/d eps_a, d eps_ab/d sigma_a,
// d sigma_ab/d sigma_a, then the same for type b; zero for the CG family of a
// pair with an ordinary type, and wherever a value is not positive (no
// derivative of a geometric mean there; relres_backward_types refuses such
// parameters).  Host only.
void install_type_params(relres_ctx* c, const double* eps_fg, const double* sig_fg,
                         const double* eps_cg, const double* sig_cg, std::vector<double>& jac)
{
    const int nt = c->ntypes;
    const size_t np = (size_t)nt * nt;
    std::vector<double> ef(np, 0.0), sf(np, 0.0), ec(np, 0.0), sc(np, 0.0);
    jac.assign(2 * np * 6, 0.0);
    const double* E[2] = {eps_fg, eps_cg};
    const double* S[2] = {sig_fg, sig_cg};
    for (int a = 0; a < nt; ++a)
        for (int b = 0; b < nt; ++b) {
            const size_t q = (size_t)a * nt + b;
            ef[q] = mix_eps(c->mix, eps_fg[a], eps_fg[b], sig_fg[a], sig_fg[b]);
            sf[q] = mix_sigma(c->mix, sig_fg[a], sig_fg[b]);
            const bool hyb = c->hybrid[a] && c->hybrid[b];
            if (hyb) {
                ec[q] = mix_eps(c->mix, eps_cg[a], eps_cg[b], sig_cg[a], sig_cg[b]);
                sc[q] = mix_sigma(c->mix, sig_cg[a], sig_cg[b]);
            }
            for (int f = 0; f < 2; ++f) {
                if (f == 1 && !hyb) continue;
                const double ea = E[f][a], eb = E[f][b], sa = S[f][a], sb = S[f][b];
                if (!(ea > 0.0 && eb > 0.0 && sa > 0.0 && sb > 0.0)) continue;
                double* J = &jac[((size_t)f * np + q) * 6];
                mix_derivs(c->mix, ea, eb, sa, sb, J);
                mix_derivs(c->mix, eb, ea, sb, sa, J + 3);
            }
        }
    build_tables(c, ef.data(), sf.data(), ec.data(), sc.data());
    c->type_par.assign(4 * (size_t)nt, 0.0);
    for (int k = 0; k < nt; ++k) {
        c->type_par[0 * nt + k] = eps_fg[k];
        c->type_par[1 * nt + k] = sig_fg[k];
        c->type_par[2 * nt + k] = eps_cg[k];
        c->type_par[3 * nt + k] = sig_cg[k];
    }
    c->tables_from_types = true;
}

// Copy the coefficient tables to the device (FP64, an FP32 copy, and the
// derivative records).  Synchronous.
int upload_tables(relres_ctx* c)
{
    std::vector<PairCoef<float>> coef32(c->coef64.size());
    for (size_t k = 0; k < coef32.size(); ++k) {
        const double* src = reinterpret_cast<const double*>(&c->coef64[k]);
        float* dst = reinterpret_cast<float*>(&coef32[k]);
        for (size_t q = 0; q < sizeof(PairCoef<double>) / sizeof(double); ++q) dst[q] = (float)src[q];
    }
    HIP_TRY(hipMemcpy(c->d_coef64.p, c->coef64.data(), sizeof(PairCoef<double>) * c->coef64.size(),
                      hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->d_coef32.p, coef32.data(), sizeof(PairCoef<float>) * coef32.size(),
                      hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->d_coef_grad.p, c->coef_grad.data(),
                      sizeof(PairCoef<double>) * c->coef_grad.size(), hipMemcpyHostToDevice));
    const size_t np = c->dist.size() / 4;
    std::vector<Cutoffs<double>> p64(np);
    std::vector<Cutoffs<float>> p32(np);
    for (size_t q = 0; q < np; ++q) {
        p64[q] = cutoffs_of<double>(&c->dist[4 * q]);
        p32[q] = cutoffs_of<float>(&c->dist[4 * q]);
    }
    HIP_TRY(hipMemcpy(c->d_pcut64.p, p64.data(), sizeof(Cutoffs<double>) * np, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->d_pcut32.p, p32.data(), sizeof(Cutoffs<float>) * np, hipMemcpyHostToDevice));
    return RELRES_OK;
}

int take_events(relres_ctx* c, hipEvent_t& a, hipEvent_t& b)
{
    for (hipEvent_t* e : {&a, &b}) {
        if (c->ev_free.empty()) {
            hipEvent_t ev;
            HIP_TRY(hipEventCreate(&ev));
            c->ev_free.push_back(ev);
        }
        *e = c->ev_free.back();
        c->ev_free.pop_back();
    }
    return RELRES_OK;
}

int next_pow2_clamped(double x, int lo, int hi)
{
    int p = 1;
    while (p < x && p < hi) p <<= 1;
    return std::max(lo, std::min(hi, p));
}

int log2i(int v)
{
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

double skin_of(const relres_ctx* c, int sy)
{
    return c->skins.empty() ? c->skin : c->skins[sy];
}

// Skin and list radii (atom list: r_s+ + skin, site list: r_c+ + skin) of
// every system.
void list_radii(const relres_ctx* c, std::vector<double>& skin, std::vector<double>& rla,
                std::vector<double>& rls)
{
    skin.resize(c->nsys);
    rla.resize(c->nsys);
    rls.resize(c->nsys);
    for (int sy = 0; sy < c->nsys; ++sy) {
        skin[sy] = skin_of(c, sy);
        rla[sy] = c->list_rso + skin[sy];
        rls[sy] = c->list_rco + skin[sy];
    }
}

// Home rows per wave of the list kernel (1 .. kRowsPerWave).  A wave tests
// its rows one after another, so a launch with few waves spreads its tests
// over more of them: when both lists together give fewer than 2048 waves at
// 8 rows, each grid takes the largest power of two that still gives it 2000
// waves.  Launches of at least 2048 waves at 16 rows take 16, so each
// stencil is loaded for as many rows as possible; the others 8.  Measured on
// MI355X: the 20480-atom liquid (3072 waves at 8 rows) builds slower with
// fewer or more rows per wave (50 µs at 8, 58 µs at 16); 6000-atom hexane
// dynamics (1000 waves) takes 5 % less time per step at 2 / 1 rows than at
// 8 / 8; the 256-replica batch (1.44 M rows) runs 3 % faster at 16 than at
// 8.  A caller override (relres_set_list_launch, relres_autotune) comes
// first; then the environment variable RELRES_LIST_ROWS="atom,site" (for
// tuning runs).
int list_rows_per_wave(bool site, long long members, long long launch_rows, int rows)
{
    if (rows >= 1 && rows <= kRowsPerWave) return rows;
    if (const char* e = std::getenv("RELRES_LIST_ROWS")) {
        int a = 0, b = 0;
        if (std::sscanf(e, "%d,%d", &a, &b) == 2) {
            const int r = site ? b : a;
            if (r >= 1 && r <= kRowsPerWave) return r;
        }
    }
    if (launch_rows >= 2048LL * 16) return 16;
    int r = 8;
    if (launch_rows >= 2048LL * r) return r;
    while (r > 1 && members < 2000LL * r) r >>= 1;
    return r;
}

// launch_rows: rows of both grids (they share the list-kernel launch);
// rows_per_wave: of the list kernel, 0 = automatic; div: cells per list
// radius (1 or 2)
int setup_grid(GridHost& g, const std::vector<double>& rl_sys, const std::vector<double>& skin_sys,
               int nsys, const double* boxes, const int* members_sys, long long launch_rows,
               int rows_per_wave, int div, long long* gen)
{
    // cells per axis of every system: a cell edge is at least the list radius
    // divided by div (with a margin far above rounding), so every pair within
    // rl lies within div cells along each axis: the 27-cell stencil (div 1)
    // or the 125-cell stencil (div 2) holds it
    std::vector<int> nn((size_t)nsys * 3);
    for (int sy = 0; sy < nsys; ++sy) {
        int* n = &nn[(size_t)sy * 3];
        long long total = 1;
        for (int k = 0; k < 3; ++k) {
            n[k] = (int)std::floor(boxes[3 * sy + k] * div / (rl_sys[sy] * (1.0 + 1e-10)));
            n[k] = std::max(1, std::min(n[k], 1023));
            total *= n[k];
        }
        while (total > (1ll << 22)) {   // keep the cell tables modest in sparse huge boxes
            total = 1;
            for (int k = 0; k < 3; ++k) {
                n[k] = std::max(1, n[k] / 2);
                total *= n[k];
            }
        }
    }
    std::vector<int> cell_base(nsys + 1, 0);
    for (int sy = 0; sy < nsys; ++sy) {
        const long long cells = (long long)nn[3 * sy] * nn[3 * sy + 1] * nn[3 * sy + 2];
        if (cell_base[sy] + cells > (1ll << 30)) return fail(RELRES_ERR_ARG, "too many cells");
        cell_base[sy + 1] = cell_base[sy] + (int)cells;
    }
    const bool same = g.nsys == nsys && g.sys_n == nn && g.rank_of_lin.p && g.div == div;
    double rl = 0.0;
    for (int sy = 0; sy < nsys; ++sy) rl = std::max(rl, rl_sys[sy]);
    g.rl = rl;
    if (!same) {
        // tables may be read by work still queued on any stream
        HIP_TRY(hipDeviceSynchronize());
        const int total = cell_base[nsys];
        std::vector<int> rank_of_lin(total), lin_of_rank(total), cell_sys(total);
        // the 27-cell stencil is tabulated; the list kernel derives the
        // 125-cell one from the cell coordinates
        std::vector<int> nbr(div == 1 ? (size_t)total * 27 : 0, -1);
        for (int sy = 0; sy < nsys; ++sy) {
            const int* n = &nn[(size_t)sy * 3];
            const int cb = cell_base[sy];
            const int nc = cell_base[sy + 1] - cb;
            std::vector<std::pair<uint32_t, int>> code(nc);
            for (int x = 0; x < n[0]; ++x)
                for (int y = 0; y < n[1]; ++y)
                    for (int z = 0; z < n[2]; ++z) {
                        const int lin = (x * n[1] + y) * n[2] + z;
                        code[lin] = {spread3(x) << 2 | spread3(y) << 1 | spread3(z), lin};
                    }
            std::sort(code.begin(), code.end());
            std::vector<int> rank(nc);
            for (int r = 0; r < nc; ++r) {
                rank[code[r].second] = r;
                lin_of_rank[cb + r] = code[r].second;
                cell_sys[cb + r] = sy;
            }
            for (int lin = 0; lin < nc; ++lin) rank_of_lin[cb + lin] = cb + rank[lin];
            if (div != 1) continue;
            // stencil ranks per cell; distinct offsets per axis (n = 1, 2 or >= 3)
            int noff[3], off[3][3];
            for (int k = 0; k < 3; ++k) {
                if (n[k] >= 3) { noff[k] = 3; off[k][0] = -1; off[k][1] = 0; off[k][2] = 1; }
                else if (n[k] == 2) { noff[k] = 2; off[k][0] = 0; off[k][1] = 1; off[k][2] = 0; }
                else { noff[k] = 1; off[k][0] = off[k][1] = off[k][2] = 0; }
            }
            for (int r = 0; r < nc; ++r) {
                const int lin = lin_of_rank[cb + r];
                const int cz = lin % n[2], cy = (lin / n[2]) % n[1], cx = lin / (n[1] * n[2]);
                for (int t = 0; t < 27; ++t) {
                    const int ix = t / 9, iy = (t / 3) % 3, iz = t % 3;
                    if (ix >= noff[0] || iy >= noff[1] || iz >= noff[2]) continue;
                    const int nx = (cx + off[0][ix] + n[0]) % n[0];
                    const int ny = (cy + off[1][iy] + n[1]) % n[1];
                    const int nz = (cz + off[2][iz] + n[2]) % n[2];
                    nbr[(size_t)(cb + r) * 27 + t] = cb + rank[(nx * n[1] + ny) * n[2] + nz];
                }
            }
        }
        TRY(ensure(g.nbr, sizeof(int) * std::max<size_t>(1, nbr.size()), gen));
        TRY(ensure(g.rank_of_lin, sizeof(int) * total, gen));
        TRY(ensure(g.lin_of_rank, sizeof(int) * total, gen));
        TRY(ensure(g.cell_sys, sizeof(int) * total, gen));
        TRY(ensure(g.count, sizeof(int) * total, gen));
        TRY(ensure(g.start, sizeof(int) * (total + 1), gen));
        if (!nbr.empty())
            HIP_TRY(hipMemcpy(g.nbr.p, nbr.data(), sizeof(int) * nbr.size(), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(g.rank_of_lin.p, rank_of_lin.data(), sizeof(int) * total, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(g.lin_of_rank.p, lin_of_rank.data(), sizeof(int) * total, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(g.cell_sys.p, cell_sys.data(), sizeof(int) * total, hipMemcpyHostToDevice));
        HIP_TRY(hipMemset(g.count.p, 0, sizeof(int) * total));
        g.nsys = nsys;
        g.sys_n = nn;
        g.div = div;
        g.ncell = total;
    }
    // rows and list-kernel waves of every grid
    long long all_members = 0;
    for (int sy = 0; sy < nsys; ++sy) all_members += members_sys[sy];
    g.rpw = list_rows_per_wave(g.site, all_members, launch_rows, rows_per_wave);
    std::vector<GeomDev> geom(nsys);
    int rows = 0, waves = 0;
    double densest = 0.0;
    for (int sy = 0; sy < nsys; ++sy) {
        GeomDev& d = geom[sy];
        std::memset(&d, 0, sizeof d);
        const double* box = boxes + 3 * sy;
        for (int k = 0; k < 3; ++k) {
            d.n[k] = nn[3 * sy + k];
            d.inv_cell[k] = d.n[k] / box[k];
            d.box[k] = box[k];
            d.half[k] = 0.5 * box[k];
        }
        d.cell_base = cell_base[sy];
        d.row_base = rows;
        d.members = members_sys[sy];
        d.wave_base = waves;
        d.rl2 = rl_sys[sy] * rl_sys[sy];
        d.half_skin2 = 0.25 * skin_sys[sy] * skin_sys[sy];
        rows += members_sys[sy];
        waves += (members_sys[sy] + g.rpw - 1) / g.rpw;
        // expected neighbours within the system's list radius
        densest = std::max(densest, members_sys[sy] / (box[0] * box[1] * box[2]) * d.rl2 * rl_sys[sy]);
    }
    g.members = rows;
    g.waves = waves;
    for (int k = 0; k < 3; ++k) g.n[k] = nn[k];
    if (geom.size() != g.geom.size() ||
        std::memcmp(geom.data(), g.geom.data(), sizeof(GeomDev) * geom.size()) != 0) {
        TRY(ensure(g.geom_dev, sizeof(GeomDev) * std::max(1, nsys), gen));
        HIP_TRY(hipDeviceSynchronize());   // the old table may still be in use
        HIP_TRY(hipMemcpy(g.geom_dev.p, geom.data(), sizeof(GeomDev) * nsys, hipMemcpyHostToDevice));
        g.geom = geom;
    }
    // the system of every list-kernel wave (with several systems), so a wave
    // finds its grid with one read instead of a search over the systems
    std::vector<int> wave_sys;
    if (nsys > 1) {
        wave_sys.resize(waves);
        for (int sy = 0; sy < nsys; ++sy)
            for (int v = geom[sy].wave_base; v < geom[sy].wave_base +
                                                 (members_sys[sy] + g.rpw - 1) / g.rpw; ++v)
                wave_sys[v] = sy;
    }
    if (wave_sys != g.wave_sys) {
        if (!wave_sys.empty()) {
            TRY(ensure(g.wave_sys_dev, sizeof(int) * wave_sys.size(), gen));
            HIP_TRY(hipDeviceSynchronize());   // the old table may still be in use
            HIP_TRY(hipMemcpy(g.wave_sys_dev.p, wave_sys.data(), sizeof(int) * wave_sys.size(),
                              hipMemcpyHostToDevice));
        }
        g.wave_sys = wave_sys;
    }
    TRY(ensure(g.user_unsorted, sizeof(int) * rows, gen));
    TRY(ensure(g.user, sizeof(int) * rows, gen));
    TRY(ensure(g.pos, sizeof(double4) * rows, gen));
    TRY(ensure(g.meta, sizeof(int2) * rows, gen));
    TRY(ensure(g.row_cell, sizeof(int) * rows, gen));
    TRY(ensure(g.nrow, sizeof(int) * rows, gen));
    if (g.cap == 0) {
        const double expect = 4.0 / 3.0 * M_PI * densest;
        g.cap = std::max(16, (int)std::ceil(expect * 1.5 + 16.0));
        g.cap = (g.cap + 7) & ~7;
    }
    TRY(ensure(g.list, sizeof(int) * (size_t)rows * g.cap, gen));

    GridDev& d = g.dev;
    d.nsys = nsys;
    d.ncell = g.ncell;
    d.members = rows;
    d.cap = g.cap;
    d.waves = waves;
    d.rows_per_wave = g.rpw;
    d.geom = g.geom_dev.as<GeomDev>();
    d.wave_sys = nsys > 1 ? g.wave_sys_dev.as<int>() : nullptr;
    d.cell_sys = g.cell_sys.as<int>();
    d.rank_of_lin = g.rank_of_lin.as<int>();
    d.lin_of_rank = g.lin_of_rank.as<int>();
    d.nbr = g.nbr.as<int>();
    d.stencil = g.div == 1 ? 3 : 5;
    d.count = g.count.as<int>();
    d.start = g.start.as<int>();
    d.user_unsorted = g.user_unsorted.as<int>();
    d.user = g.user.as<int>();
    d.pos = g.pos.as<double4>();
    d.meta = g.meta.as<int2>();
    d.row_cell = g.row_cell.as<int>();
    d.list = g.list.as<int>();
    d.nrow = g.nrow.as<int>();
    return RELRES_OK;
}

// Bucket slots per cell for the one-launch placement: room for about twice
// the mean occupancy plus 8, a power of two of at most 64 (0: the grid's cells
// are too crowded for buckets).
int bucket_slots(const GridHost& g)
{
    if (g.ncell <= 0) return 0;
    const double mean = (double)g.members / g.ncell;
    int cap = 8;
    while (cap < 2.0 * mean + 8.0 && cap <= 64) cap *= 2;
    return cap <= 64 ? cap : 0;
}

// Sets both grids' bucket capacity: buckets for all grids or for none.
int set_buckets(relres_ctx* c, GridHost& ga, GridHost* gs, bool want, bool* used)
{
    int cap_a = want ? bucket_slots(ga) : 0;
    int cap_s = (want && gs) ? bucket_slots(*gs) : 0;
    const bool use = cap_a > 0 && (!gs || cap_s > 0);
    if (!use) cap_a = cap_s = 0;
    if (cap_a > 0) TRY(ensure(ga.user_unsorted, sizeof(int) * (size_t)ga.ncell * cap_a, &c->alloc_generation));
    ga.dev.bucket_cap = cap_a;
    ga.dev.user_unsorted = ga.user_unsorted.as<int>();
    if (gs) {
        if (cap_s > 0)
            TRY(ensure(gs->user_unsorted, sizeof(int) * (size_t)gs->ncell * cap_s, &c->alloc_generation));
        gs->dev.bucket_cap = cap_s;
        gs->dev.user_unsorted = gs->user_unsorted.as<int>();
    }
    *used = use;
    return RELRES_OK;
}

TopoDev topo_of(relres_ctx* c)
{
    TopoDev t;
    t.types = c->d_types.as<int>();
    t.mol = c->d_mol.as<int>();
    t.hybrid = c->d_hybrid.as<int>();
    t.excl_off = c->has_excl ? c->d_excl_off.as<int>() : nullptr;
    t.excl_idx = c->has_excl ? c->d_excl_idx.as<int>() : nullptr;
    t.same_mol = c->same_mol;
    t.n = c->n;
    t.max_excl = c->max_excl;
    t.sys = c->nsys > 1 ? c->d_sys.as<int>() : nullptr;
    return t;
}

// Copy the grid descriptors to the device when they changed since the last
// upload (new box, cell counts, capacities or buffers).  The pinned staging
// buffer is rewritten only once the previous upload from it has completed.
int upload_grids(relres_ctx* c, hipStream_t s)
{
    GridDev want[2] = {c->ga.dev, c->n_sites > 0 ? c->gs.dev : c->ga.dev};
    if (c->grids_valid && std::memcmp(want, c->uploaded, sizeof want) == 0) return RELRES_OK;
    if (c->upload_pending) HIP_TRY(hipEventSynchronize(c->ev_upload));
    std::memcpy(c->h_grids, want, sizeof want);
    HIP_TRY(hipMemcpyAsync(c->d_grids.p, c->h_grids, sizeof want, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(c->ev_upload, s));
    c->upload_pending = true;
    std::memcpy(c->uploaded, want, sizeof want);
    c->grids_valid = true;
    return RELRES_OK;
}

// Exact entries and longest rows of both lists (one small kernel, then a
// synchronisation); refreshes the statistics and the automatic lane counts.
int refresh_list_stats(relres_ctx* c, hipStream_t s)
{
    const bool sites = c->n_sites > 0;
    if (c->n > 0) {
        HIP_TRY(launch_list_stats(c->d_grids.as<GridDev>(), sites ? 2 : 1, c->d_status.as<Status>(), s));
        HIP_TRY(hipMemcpyAsync(c->h_status, c->d_status.p, sizeof(Status), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    relres_stats& st = c->stats;
    st.atom_entries = c->n ? (long long)c->h_status->entries[0] : 0;
    st.site_entries = (c->n && sites) ? (long long)c->h_status->entries[1] : 0;
    st.atom_max_row = c->n ? c->h_status->longest[0] : 0;
    st.site_max_row = (c->n && sites) ? c->h_status->longest[1] : 0;
    // Automatic lanes per row: about E list entries per lane.  A launch that
    // fits the machine a few times over is latency-bound and takes E = 4
    // (short chains per lane); a much larger one is bound by issue, and its
    // per-row work (record, reductions across the row's lanes) shrinks with
    // fewer lanes per row: E = 8, then 16.  Measured on MI355X (force launch):
    // the 20480-atom liquid (2304 waves at E = 4) is fastest at E = 4; the
    // 98304-atom copolymer (24576 waves) at E = 8, 38.4 against 45.9 us; the
    // 256-replica batch (210000 waves) at E = 16, 221 against 342 us.
    const double avg_a = c->n ? (double)st.atom_entries / c->n : 0.0;
    const double avg_s = c->n_sites ? (double)st.site_entries / c->n_sites : 0.0;
    const long long waves4 =
        ((long long)c->n * next_pow2_clamped(avg_a / 4.0, 1, 32) +
         (long long)c->n_sites * next_pow2_clamped((avg_a + avg_s) / 4.0, 1, 64)) / 64;
    const double per_lane = waves4 <= 8192 ? 4.0 : (waves4 <= 65536 ? 8.0 : 16.0);
    c->auto_la = next_pow2_clamped(avg_a / per_lane, 1, 32);
    c->auto_lb = next_pow2_clamped((avg_a + avg_s) / per_lane, 1, 64);
    c->stats_fresh = true;
    return RELRES_OK;
}

// List builder: groups of rows per wave.  One block per cell remains
// available with RELRES_LIST_KERNEL=block; it is slower at every occupancy
// measured (94 atoms per cell: 790 us against 72 us per build), because a
// grid of few, crowded cells gives it few blocks.
bool lists_per_wave(const relres_ctx* c)
{
    (void)c;
    if (const char* e = std::getenv("RELRES_LIST_KERNEL"))
        if (!std::strcmp(e, "block")) return false;
    return true;
}

// Enqueue one list build on `s`: bin, scan, scatter, cell sort, lists, then
// (unless the stream is being captured) a copy of the status word to pinned
// host memory and an event.  Nothing waits;
// relres_forces may be enqueued behind it at once.  The lists are complete
// unless examine_status() later reports an overflow.
int enqueue_build(relres_ctx* c, const double* pos, const double* box, hipStream_t s)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    if (!c->topo_set) return fail(RELRES_ERR_STATE, "relres_set_topology has not been called");
    if (!box) return fail(RELRES_ERR_ARG, "box is NULL");
    if (c->n > 0 && !pos) return fail(RELRES_ERR_ARG, "pos is NULL");
    const int ns = c->nsys;
    for (int k = 0; k < 3 * ns; ++k)
        if (!(std::isfinite(box[k]) && box[k] > 0.0))
            return fail(RELRES_ERR_ARG, "bad box edge %g (system %d)", box[k], k / 3);
    std::vector<double> skin_sys, rla, rls;
    list_radii(c, skin_sys, rla, rls);
    const bool sites = c->n_sites > 0;
    for (int sy = 0; sy < ns; ++sy) {
        // a system without hybrid atoms only needs the atom-list radius
        const double rmax = c->sites_sys[sy] > 0 ? rls[sy] : rla[sy];
        for (int k = 0; k < 3; ++k)
            if (!(box[3 * sy + k] > 2.0 * rmax))
                return fail(RELRES_ERR_BOX_TOO_SMALL, "box edge %g of system %d must exceed 2 x %g",
                            box[3 * sy + k], sy, rmax);
    }
    c->built = false;
    // positions of the previous build are comparable when the boxes and skins are the same
    const bool same_boxes = c->boxes.size() == (size_t)3 * ns &&
                            std::equal(box, box + 3 * ns, c->boxes.begin()) && c->ref_skins == skin_sys;
    std::copy(box, box + 3, c->box);
    c->boxes.assign(box, box + 3 * ns);
    {
        std::vector<double> bd((size_t)6 * ns);
        for (int sy = 0; sy < ns; ++sy)
            for (int k = 0; k < 3; ++k) {
                bd[6 * sy + k] = box[3 * sy + k];
                bd[6 * sy + 3 + k] = 1.0 / box[3 * sy + k];
            }
        if (bd != c->boxes_dev) {
            TRY(ensure(c->d_boxes, sizeof(double) * bd.size(), &c->alloc_generation));
            HIP_TRY(hipDeviceSynchronize());   // the old values may still be in use
            HIP_TRY(hipMemcpy(c->d_boxes.p, bd.data(), sizeof(double) * bd.size(), hipMemcpyHostToDevice));
            c->boxes_dev = bd;
        }
    }
    const int dims_before = c->ga.ncell + (sites ? c->gs.ncell : 0);
    const long long launch_rows = (long long)c->n + c->n_sites;
    TRY(setup_grid(c->ga, rla, skin_sys, ns, box, c->atoms_sys.data(), launch_rows, c->rows_a,
                   c->div_a ? c->div_a : 1, &c->alloc_generation));
    if (sites)
        TRY(setup_grid(c->gs, rls, skin_sys, ns, box, c->sites_sys.data(), launch_rows, c->rows_s,
                       c->div_s ? c->div_s : 1, &c->alloc_generation));
    if (c->ga.ncell + (sites ? c->gs.ncell : 0) != dims_before) c->lanes_stale = true;
    bool one_launch = false;
    TRY(set_buckets(c, c->ga, sites ? &c->gs : nullptr,
                    c->place_one_launch && c->ga.ncell + (sites ? c->gs.ncell : 0) <= kPlaceMaxCells,
                    &one_launch));
    const void* wpos_before = c->d_wpos.p;
    TRY(ensure(c->d_wpos, sizeof(double4) * c->n, &c->alloc_generation));
    const bool check_moved = c->ref_valid && same_boxes && c->d_wpos.p == wpos_before;
    TRY(ensure(c->d_key_a, sizeof(int2) * c->n, &c->alloc_generation));
    TRY(ensure(c->d_key_s, sizeof(int2) * c->n, &c->alloc_generation));
    TRY(ensure(c->d_user2arow, sizeof(int) * c->n, &c->alloc_generation));
    TRY(ensure(c->d_seg_tot, sizeof(int) * (size_t)(scan_segments(c->ga.ncell) +
                                                   (sites ? scan_segments(c->gs.ncell) : 0) + 1),
               &c->alloc_generation));
    TRY(ensure(c->d_a_rec, sizeof(int4) * std::max(1, c->n), &c->alloc_generation));
    TRY(ensure(c->d_s_rec, sizeof(int4) * std::max(1, c->n_sites), &c->alloc_generation));

    hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &capture));
    const bool capturing = capture != hipStreamCaptureStatusNone;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timed = c->timing && !capturing;
    if (timed) {
        TRY(take_events(c, e0, e1));
        HIP_TRY(hipEventRecord(e0, s));
    }
    if (c->n > 0) {
        TRY(upload_grids(c, s));
        const TopoDev topo = topo_of(c);
        GridDev* gd = c->d_grids.as<GridDev>();
        HIP_TRY(launch_bin(c->n, pos, topo, gd, c->d_wpos.as<double4>(), c->d_key_a.as<int2>(),
                           c->d_key_s.as<int2>(), c->d_status.as<Status>(), check_moved, s));
        c->ref_valid = true;
        c->ref_skins = skin_sys;
        const int ncs = sites ? c->gs.ncell : 0;
        const long long members = (long long)c->n + (sites ? c->n_sites : 0);
        if (one_launch) {
            HIP_TRY(launch_place(gd, c->ga.ncell, ncs, members, c->n, c->d_key_a.as<int2>(),
                                 c->d_key_s.as<int2>(), c->d_wpos.as<double4>(), topo,
                                 c->d_user2arow.as<int>(), s));
        } else {
            HIP_TRY(launch_scan(gd, sites ? 2 : 1, c->ga.ncell, ncs, c->d_seg_tot.as<int>(), s));
            HIP_TRY(launch_scatter(c->n, gd, c->d_key_a.as<int2>(), c->d_key_s.as<int2>(), s));
            HIP_TRY(launch_cellsort(gd, c->ga.ncell, c->ga.ncell + ncs, members,
                                    c->d_wpos.as<double4>(), topo, c->d_user2arow.as<int>(), s));
        }
        HIP_TRY(launch_lists(gd, c->ga.ncell, ncs, c->ga.waves, sites ? c->gs.waves : 0, topo,
                             c->d_user2arow.as<int>(),
                             c->d_a_rec.as<int4>(), c->d_s_rec.as<int4>(),
                             c->d_status.as<Status>(), lists_per_wave(c), c->cand,
                             c->ga.div == 2 ? 5 : 3, (sites && c->gs.div == 2) ? 5 : 3, s));
        // A captured build copies nothing: the status only accumulates (see
        // Status), so relres_check_lists copies it once after the caller has
        // synchronised, covering every replay since the previous check.
        if (!capturing) {
            HIP_TRY(hipMemcpyAsync(c->h_status, c->d_status.p, sizeof(Status), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipEventRecord(c->ev_status, s));
        }
        c->status_in_graph = capturing;
        c->check_pending = true;
    }
    if (timed) {
        HIP_TRY(hipEventRecord(e1, s));
        c->ev_build.push_back({e0, e1});
    }
    relres_stats& st = c->stats;
    st.n_atoms = c->n;
    st.n_sites = c->n_sites;
    if (c->n > 0) st.place_launches = one_launch ? 1 : 3;
    for (int k = 0; k < 3; ++k) {
        st.atom_cells[k] = c->ga.n[k];
        st.site_cells[k] = sites ? c->gs.n[k] : 0;
        st.box[k] = box[k];
    }
    st.builds++;
    c->stats_fresh = false;
    c->built = true;
    return RELRES_OK;
}

// RELRES_ERR_EW_TIMEOUT once for force calls whose energy/virial wait gave up
// since the previous examination (h_status must be current).
int take_ew_failures(relres_ctx* c)
{
    const unsigned f = c->h_status->ew_failed;
    if (f == c->ew_failed_seen) return RELRES_OK;
    c->ew_failed_seen = f;
    return fail(RELRES_ERR_EW_TIMEOUT, "an energy/virial reduction gave up waiting for other "
                "blocks; the energy and virial of that call are NaN");
}

// Make h_status describe the last enqueued build: wait for its copy, or, for
// a build captured into a graph (the caller has synchronised after the
// replays), copy the accumulated status now.
int fetch_status(relres_ctx* c)
{
    if (c->status_in_graph)
        HIP_TRY(hipMemcpy(c->h_status, c->d_status.p, sizeof(Status), hipMemcpyDeviceToHost));
    else
        HIP_TRY(hipEventSynchronize(c->ev_status));
    return RELRES_OK;
}

// Wait for the status of the last enqueued build and examine it.  Returns
// RELRES_OK (lists complete), RELRES_ERR_NONFINITE, or RELRES_ERR_LIST_RETRY
// after growing the capacities of the rows that overflowed (the lists are
// then invalid until the next build).
int examine_status(relres_ctx* c)
{
    // a build captured in a graph is examined at every check (each replay
    // rebuilds the lists and copies a new status)
    if (!c->check_pending && !c->status_in_graph)
        return c->built ? RELRES_OK : fail(RELRES_ERR_NO_LISTS, "no lists");
    TRY(fetch_status(c));
    c->check_pending = false;
    const Status& st = *c->h_status;
    const unsigned moved = st.moved - c->moved_seen;
    c->moved_seen = st.moved;
    if (st.nonfinite != c->nonfinite_seen) {
        c->nonfinite_seen = st.nonfinite;
        c->built = false;
        c->ref_valid = false;
        return fail(RELRES_ERR_NONFINITE, "non-finite position");
    }
    c->stats.moved_at_last_build = moved;
    if (moved > 0) {
        c->stats.dangerous_builds++;
        c->warn_pending = true;
    }
    const bool sites = c->n_sites > 0;
    const int mr_a = st.max_row[0], mr_s = st.max_row[1];
    const bool ov_a = mr_a > c->ga.cap;
    const bool ov_s = sites && mr_s > c->gs.cap;
    if (!ov_a && !ov_s) return RELRES_OK;
    if (ov_a) {
        c->ga.cap = ((int)(mr_a * 1.25) + 8 + 7) & ~7;
        std::vector<double> skin_sys, rla, rls;
        list_radii(c, skin_sys, rla, rls);
        TRY(setup_grid(c->ga, rla, skin_sys, c->nsys, c->boxes.data(), c->atoms_sys.data(),
                       (long long)c->n + c->n_sites, c->rows_a, c->ga.div, &c->alloc_generation));
    }
    if (ov_s) {
        c->gs.cap = ((int)(mr_s * 1.25) + 8 + 7) & ~7;
        std::vector<double> skin_sys, rla, rls;
        list_radii(c, skin_sys, rla, rls);
        TRY(setup_grid(c->gs, rls, skin_sys, c->nsys, c->boxes.data(), c->sites_sys.data(),
                       (long long)c->n + c->n_sites, c->rows_s, c->gs.div, &c->alloc_generation));
    }
    c->stats.regrows++;
    c->lanes_stale = true;
    c->built = false;
    return fail(RELRES_ERR_LIST_RETRY, "list rows overflowed (atom %d/%d, site %d/%d); capacity grown",
                mr_a, c->ga.cap, mr_s, sites ? c->gs.cap : 0);
}

// Consume a pending status before a new build replaces it: an overflow only
// matters for its capacity growth, which examine_status already applied.
int drain_check(relres_ctx* c)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    // the status of a captured build describes replays, which only
    // relres_check_lists examines (it copies the status, which must not
    // happen while a stream is being captured)
    if (c->status_in_graph) {
        c->check_pending = false;
        return RELRES_OK;
    }
    const int rc = examine_status(c);
    return (rc == RELRES_ERR_LIST_RETRY || rc == RELRES_ERR_NO_LISTS) ? RELRES_OK : rc;
}

// Build, wait, and rebuild with grown rows until the lists are complete.
int build_checked(relres_ctx* c, const double* pos, const double* box, hipStream_t s)
{
    TRY(drain_check(c));
    int rc = RELRES_ERR_LIST_RETRY;
    for (int attempt = 0; attempt < 4 && rc == RELRES_ERR_LIST_RETRY; ++attempt) {
        TRY(enqueue_build(c, pos, box, s));
        rc = examine_status(c);
    }
    if (rc == RELRES_ERR_LIST_RETRY) return fail(RELRES_ERR_LIST_OVERFLOW, "list capacity did not converge");
    if (rc != RELRES_OK) return rc;
    relres_stats& st = c->stats;
    st.atom_capacity = c->ga.cap;
    st.site_capacity = c->n_sites > 0 ? c->gs.cap : 0;
    if (c->lanes_stale) {
        TRY(refresh_list_stats(c, s));
        c->lanes_stale = false;
    }
    return RELRES_OK;
}

// RELRES_WARN_DANGEROUS_BUILD once for every build that found atoms more than
// half the skin from their previous-build positions (lists complete).
int take_warning(relres_ctx* c)
{
    if (!c->warn_pending) return RELRES_OK;
    c->warn_pending = false;
    return RELRES_WARN_DANGEROUS_BUILD;
}

// Device address of `scratch` on the current device, looked up once per
// device (the array has one copy per GPU, at its own address).
int scratch_of_device(int device, void** out, hipError_t* err)
{
    static std::mutex mu;
    static std::vector<void*> addr;
    static std::vector<hipError_t> errs;
    std::lock_guard<std::mutex> lock(mu);
    if (device < 0) return RELRES_ERR_ARG;
    if ((size_t)device >= addr.size()) {
        addr.resize(device + 1, nullptr);
        errs.resize(device + 1, hipSuccess);
    }
    if (!addr[device] && errs[device] == hipSuccess) {
        void* p = nullptr;
        const hipError_t e = scratch_address(&p);
        if (e != hipSuccess || !p) errs[device] = e != hipSuccess ? e : hipErrorInvalidSymbol;
        else addr[device] = p;
    }
    *out = addr[device];
    *err = errs[device];
    return RELRES_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

int relres_abi_version(void) { return RELRES_ABI_VERSION; }

double relres_mix_distance(int mix, double a, double b)
{
    if (mix != RELRES_MIX_GEOMETRIC && mix != RELRES_MIX_ARITHMETIC && mix != RELRES_MIX_SIXTHPOWER)
        return std::numeric_limits<double>::quiet_NaN();
    return mix_sigma(mix, a, b);
}

// Eq. 15 (one CG site from its FG sites, geometric FG mixing) and Eq. 13 (a
// pair of CG sites from all FG pair parameters between them).
int relres_cg_site_params(int n, const double* eps_fg, const double* sig_fg, double* eps_cg,
                          double* sig_cg)
{
    if (n < 1 || !eps_fg || !sig_fg || !eps_cg || !sig_cg) return fail(RELRES_ERR_ARG, "bad argument");
    double b12 = 0.0, b6 = 0.0;
    for (int k = 0; k < n; ++k) {
        const double e = eps_fg[k], sg = sig_fg[k];
        if (!(std::isfinite(e) && e >= 0.0 && std::isfinite(sg) && sg > 0.0))
            return fail(RELRES_ERR_ARG, "bad FG parameters of site %d", k);
        const double s3 = sg * sg * sg;
        const double se = std::sqrt(e);
        b12 += se * s3 * s3;          // sqrt(eps sigma^12)
        b6 += se * s3;                // sqrt(eps sigma^6)
    }
    if (!(b6 > 0.0)) return fail(RELRES_ERR_ARG, "all FG energies are zero");
    *sig_cg = std::cbrt(b12 / b6);
    *eps_cg = (b6 * b6) * (b6 * b6) / (b12 * b12);
    return RELRES_OK;
}

int relres_cg_pair_params(int n, const double* eps_mn, const double* sig_mn, double* eps_cg,
                          double* sig_cg)
{
    if (n < 1 || !eps_mn || !sig_mn || !eps_cg || !sig_cg) return fail(RELRES_ERR_ARG, "bad argument");
    double a12 = 0.0, a6 = 0.0;
    for (int k = 0; k < n; ++k) {
        const double e = eps_mn[k], sg = sig_mn[k];
        if (!(std::isfinite(e) && e >= 0.0 && std::isfinite(sg) && sg > 0.0))
            return fail(RELRES_ERR_ARG, "bad FG pair parameters at %d", k);
        const double s6 = (sg * sg * sg) * (sg * sg * sg);
        a12 += e * s6 * s6;
        a6 += e * s6;
    }
    if (!(a6 > 0.0)) return fail(RELRES_ERR_ARG, "all FG energies are zero");
    *sig_cg = std::pow(a12 / a6, 1.0 / 6.0);
    *eps_cg = a6 * a6 / a12;
    return RELRES_OK;
}

const char* relres_last_error(void) { return g_last_error.c_str(); }

const char* relres_strerror(int code)
{
    switch (code) {
    case RELRES_OK: return "ok";
    case RELRES_ERR_ARG: return "invalid argument";
    case RELRES_ERR_CUTOFF_ORDER: return "cutoffs must satisfy r_s- <= r_s+ <= r_c- <= r_c+ (and skin >= 0)";
    case RELRES_ERR_BOX_TOO_SMALL: return "box edge not larger than twice the list radius";
    case RELRES_ERR_TOPOLOGY: return "invalid topology";
    case RELRES_ERR_HIP: return "HIP runtime error";
    case RELRES_ERR_NO_LISTS: return "no neighbour lists: call relres_build_lists first";
    case RELRES_ERR_LIST_OVERFLOW: return "neighbour list capacity could not be grown";
    case RELRES_ERR_NONFINITE: return "non-finite position";
    case RELRES_ERR_STATE: return "call out of order";
    case RELRES_ERR_LIST_RETRY: return "neighbour lists overflowed: capacity grown, build again";
    case RELRES_ERR_STALE_LISTS: return "an atom moved more than half the skin since the last list build";
    case RELRES_ERR_EW_TIMEOUT: return "a force call gave up waiting for its energy/virial sums (they are NaN)";
    case RELRES_WARN_DANGEROUS_BUILD: return "warning: atoms had moved more than half the skin since the previous build";
    default: return "unknown error";
    }
}

int relres_create(const relres_params* p, relres_ctx** out)
{
    if (!out) return fail(RELRES_ERR_ARG, "out is NULL");
    *out = nullptr;
    if (!p) return fail(RELRES_ERR_ARG, "params is NULL");
    if (p->ntypes < 1 || p->ntypes > RELRES_MAX_TYPES)
        return fail(RELRES_ERR_ARG, "ntypes %d outside [1, %d]", p->ntypes, RELRES_MAX_TYPES);
    if (!p->eps_fg || !p->sig_fg || !p->eps_cg || !p->sig_cg)
        return fail(RELRES_ERR_ARG, "per-type parameter array is NULL");
    if (p->precision != 32 && p->precision != 64)
        return fail(RELRES_ERR_ARG, "precision must be 32 or 64");
    if (p->pair_math != 0 && p->pair_math != 32 && p->pair_math != 64)
        return fail(RELRES_ERR_ARG, "pair_math must be 0, 32 or 64");
    if (p->precision == 64 && p->pair_math == 32)
        return fail(RELRES_ERR_ARG, "FP64 forces need FP64 pair terms");
    if (p->mix != RELRES_MIX_GEOMETRIC && p->mix != RELRES_MIX_ARITHMETIC &&
        p->mix != RELRES_MIX_SIXTHPOWER)
        return fail(RELRES_ERR_ARG, "unknown mixing rule %d", p->mix);
    if (p->no_shift != 0 && p->no_shift != 1) return fail(RELRES_ERR_ARG, "no_shift must be 0 or 1");
    const double cut[5] = {p->rs_in, p->rs_out, p->rc_in, p->rc_out, p->skin};
    for (double v : cut)
        if (!std::isfinite(v)) return fail(RELRES_ERR_CUTOFF_ORDER, "non-finite cutoff");
    if (!(0.0 < p->rs_in && p->rs_in <= p->rs_out && p->rs_out <= p->rc_in &&
          p->rc_in <= p->rc_out && p->skin >= 0.0))
        return fail(RELRES_ERR_CUTOFF_ORDER, "need 0 < r_s- <= r_s+ <= r_c- <= r_c+, skin >= 0 "
                    "(got %g %g %g %g, skin %g)", p->rs_in, p->rs_out, p->rc_in, p->rc_out, p->skin);
    const int nt = p->ntypes;
    for (int t = 0; t < nt; ++t) {
        if (!(std::isfinite(p->eps_fg[t]) && p->eps_fg[t] >= 0.0 && std::isfinite(p->sig_fg[t]) &&
              p->sig_fg[t] > 0.0))
            return fail(RELRES_ERR_ARG, "bad FG parameters for type %d", t);
        if (!(std::isfinite(p->eps_cg[t]) && p->eps_cg[t] >= 0.0 && std::isfinite(p->sig_cg[t])))
            return fail(RELRES_ERR_ARG, "bad CG parameters for type %d", t);
        if (p->eps_cg[t] > 0.0 && !(p->sig_cg[t] > 0.0))
            return fail(RELRES_ERR_ARG, "hybrid type %d needs sigma_CG > 0", t);
    }

    // distances of every type pair: explicit, mixed from per-type values
    // (each distance with the sigma rule; like types keep their own), or global
    std::vector<double> dist((size_t)4 * nt * nt);
    for (int a = 0; a < nt; ++a)
        for (int b = 0; b < nt; ++b)
            for (int k = 0; k < 4; ++k) {
                const size_t q = (size_t)a * nt + b;
                double v = cut[k];
                if (p->cut_pair) v = p->cut_pair[4 * q + k];
                else if (p->cut_type && a == b) v = p->cut_type[4 * a + k];
                else if (p->cut_type) v = mix_sigma(p->mix, p->cut_type[4 * a + k], p->cut_type[4 * b + k]);
                dist[4 * q + k] = v;
            }
    for (int a = 0; a < nt; ++a)
        for (int b = 0; b < nt; ++b) {
            const double* r = &dist[4 * ((size_t)a * nt + b)];
            const double* rt = &dist[4 * ((size_t)b * nt + a)];
            if (!(std::isfinite(r[0]) && std::isfinite(r[3]) && 0.0 < r[0] && r[0] <= r[1] &&
                  r[1] <= r[2] && r[2] <= r[3]))
                return fail(RELRES_ERR_CUTOFF_ORDER, "type pair (%d, %d): need 0 < r_s- <= r_s+ <= "
                            "r_c- <= r_c+ (got %g %g %g %g)", a, b, r[0], r[1], r[2], r[3]);
            if (!std::equal(r, r + 4, rt))
                return fail(RELRES_ERR_ARG, "cut_pair is not symmetric for types (%d, %d)", a, b);
        }

    relres_ctx* c = new relres_ctx();
    c->gs.site = true;
    auto bail = [&](int rc) { relres_destroy(c); return rc; };
    if (hipGetDevice(&c->device) != hipSuccess) return bail(fail(RELRES_ERR_HIP, "no HIP device"));
    // the static scratch of relres_forces_noalloc, once per device (a failure
    // only disables that entry point, which reports it)
    if (scratch_of_device(c->device, &c->scratch, &c->scratch_err) != RELRES_OK)
        return bail(fail(RELRES_ERR_HIP, "bad device %d", c->device));
    c->skin = p->skin;
    // RELRES_EW_SPIN_LIMIT: polls of a cross-block energy/virial wait before it
    // gives up (a negative value gives up at once: failure handling tests)
    if (const char* e = std::getenv("RELRES_EW_SPIN_LIMIT")) c->spin_limit = std::atoi(e);
    // RELRES_PLACE=classic: the scan / scatter / cell-sort launches for every
    // grid (the one-launch placement is then never used; parity tests of both)
    if (const char* e = std::getenv("RELRES_PLACE"))
        c->place_one_launch = std::strcmp(e, "classic") != 0;
    c->ntypes = nt;
    c->mix = p->mix;
    c->no_shift = p->no_shift;
    c->precision = p->precision;
    c->pair_math = p->pair_math ? p->pair_math : p->precision;
    c->hybrid.resize(nt);
    for (int t = 0; t < nt; ++t) c->hybrid[t] = p->eps_cg[t] > 0.0 ? 1 : 0;
    c->dist = dist;
    c->per_pair = false;
    c->list_rso = c->list_rco = 0.0;
    double any_rco = 0.0;
    for (int a = 0; a < nt; ++a)
        for (int b = 0; b < nt; ++b) {
            const double* r = &dist[4 * ((size_t)a * nt + b)];
            if (!std::equal(r, r + 4, &dist[0])) c->per_pair = true;
            c->list_rso = std::max(c->list_rso, r[1]);
            any_rco = std::max(any_rco, r[3]);
            if (c->hybrid[a] && c->hybrid[b]) c->list_rco = std::max(c->list_rco, r[3]);
        }
    if (c->list_rco == 0.0) c->list_rco = any_rco;     // no hybrid pair: the site list stays empty

    std::vector<double> jac;
    install_type_params(c, p->eps_fg, p->sig_fg, p->eps_cg, p->sig_cg, jac);
    for (int k = 0; k < 4; ++k) c->cut64[k] = dist[k];
    for (int k = 0; k < 4; ++k) c->cut64[4 + k] = c->cut64[k] * c->cut64[k];

    int rc;
    if ((rc = ensure(c->d_coef64, sizeof(PairCoef<double>) * c->coef64.size(), &c->alloc_generation))) return bail(rc);
    if ((rc = ensure(c->d_coef32, sizeof(PairCoef<float>) * c->coef64.size(), &c->alloc_generation))) return bail(rc);
    if ((rc = ensure(c->d_coef_grad, sizeof(PairCoef<double>) * c->coef_grad.size(), &c->alloc_generation))) return bail(rc);
    if ((rc = ensure(c->d_pcut64, sizeof(Cutoffs<double>) * nt * nt, &c->alloc_generation))) return bail(rc);
    if ((rc = ensure(c->d_pcut32, sizeof(Cutoffs<float>) * nt * nt, &c->alloc_generation))) return bail(rc);
    if ((rc = ensure(c->d_hybrid, sizeof(int) * nt, &c->alloc_generation))) return bail(rc);
    if ((rc = ensure(c->d_mix_jac, sizeof(double) * jac.size(), &c->alloc_generation))) return bail(rc);
    if ((rc = ensure(c->d_gpair, sizeof(double) * 4 * nt * nt, &c->alloc_generation))) return bail(rc);
    if ((rc = ensure(c->d_grids, 2 * sizeof(GridDev), &c->alloc_generation))) return bail(rc);
    if ((rc = ensure(c->d_status, sizeof(Status), &c->alloc_generation))) return bail(rc);
    if ((rc = ensure(c->d_epoch, 256, &c->alloc_generation))) return bail(rc);
    if (upload_tables(c) != RELRES_OK ||
        hipMemcpy(c->d_hybrid.p, c->hybrid.data(), sizeof(int) * nt, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->d_mix_jac.p, jac.data(), sizeof(double) * jac.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(c->d_status.p, 0, sizeof(Status)) != hipSuccess ||
        hipMemset(c->d_epoch.p, 0, 256) != hipSuccess)
        return bail(fail(RELRES_ERR_HIP, "uploading parameters failed"));
    if (hipHostMalloc((void**)&c->h_grids, 2 * sizeof(GridDev), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->h_status, sizeof(Status), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&c->h_query, sizeof(Status), hipHostMallocDefault) != hipSuccess)
        return bail(fail(RELRES_ERR_HIP, "pinned host allocation failed"));
    if (hipEventCreateWithFlags(&c->ev_status, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_upload, hipEventDisableTiming) != hipSuccess)
        return bail(fail(RELRES_ERR_HIP, "event creation failed"));
    std::memset(c->h_grids, 0, 2 * sizeof(GridDev));
    std::memset(c->h_status, 0, sizeof(Status));
    std::memset(c->h_query, 0, sizeof(Status));
    *out = c;
    return RELRES_OK;
}

int relres_set_topology(relres_ctx* c, int n, const int* types, const int* mol, int exclude_same_mol,
                        const int* excl_offsets, const int* excl_idx)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    if (n < 0 || n >= RELRES_MAX_ATOMS) return fail(RELRES_ERR_ARG, "n_atoms %d out of range", n);
    if (n > 0 && !types) return fail(RELRES_ERR_ARG, "types is NULL");
    if (exclude_same_mol && n > 0 && !mol) return fail(RELRES_ERR_ARG, "mol is NULL");
    std::vector<int> t(types, types + n), m(n, 0);
    if (mol) std::copy(mol, mol + n, m.begin());
    int sites = 0;
    for (int i = 0; i < n; ++i) {
        if (t[i] < 0 || t[i] >= c->ntypes)
            return fail(RELRES_ERR_TOPOLOGY, "type %d of atom %d outside [0, %d)", t[i], i, c->ntypes);
        sites += c->hybrid[t[i]];
    }
    // exclusions: validate, symmetrise, sort, deduplicate
    std::vector<int> off(n + 1, 0), idx;
    if (excl_offsets && n > 0) {
        if (excl_offsets[0] != 0) return fail(RELRES_ERR_TOPOLOGY, "excl_offsets[0] != 0");
        for (int i = 0; i < n; ++i)
            if (excl_offsets[i + 1] < excl_offsets[i])
                return fail(RELRES_ERR_TOPOLOGY, "excl_offsets decrease at %d", i);
        if (excl_offsets[n] > 0 && !excl_idx) return fail(RELRES_ERR_TOPOLOGY, "excl_idx is NULL");
        std::vector<std::vector<int>> part(n);
        for (int i = 0; i < n; ++i)
            for (int k = excl_offsets[i]; k < excl_offsets[i + 1]; ++k) {
                const int j = excl_idx[k];
                if (j < 0 || j >= n || j == i)
                    return fail(RELRES_ERR_TOPOLOGY, "bad exclusion %d of atom %d", j, i);
                part[i].push_back(j);
                part[j].push_back(i);
            }
        for (int i = 0; i < n; ++i) {
            std::sort(part[i].begin(), part[i].end());
            part[i].erase(std::unique(part[i].begin(), part[i].end()), part[i].end());
            if ((int)part[i].size() > RELRES_MAX_EXCLUSIONS)
                return fail(RELRES_ERR_TOPOLOGY, "atom %d has %d excluded partners (max %d)", i,
                            (int)part[i].size(), RELRES_MAX_EXCLUSIONS);
            off[i + 1] = off[i] + (int)part[i].size();
            idx.insert(idx.end(), part[i].begin(), part[i].end());
        }
    }
    if (c->check_pending || c->status_in_graph) {
        // a build of the previous topology (or replays of a captured one)
        // is still unexamined: retire it
        TRY(fetch_status(c));
        c->nonfinite_seen = c->h_status->nonfinite;
        c->moved_seen = c->h_status->moved;
        c->check_pending = false;
    }
    c->ref_valid = false;
    c->warn_pending = false;
    c->built = false;
    c->topo_set = false;
    c->lanes_stale = true;
    c->n = n;
    c->n_sites = sites;
    c->h_types = t;
    c->nsys = 1;                      // one system until relres_set_systems says otherwise
    c->skins.clear();
    c->sys_off = {0, n};
    c->atoms_sys = {n};
    c->sites_sys = {sites};
    c->same_mol = exclude_same_mol ? 1 : 0;
    c->has_excl = !idx.empty();
    c->max_excl = 0;
    for (int i = 0; i < n; ++i) c->max_excl = std::max(c->max_excl, off[i + 1] - off[i]);
    TRY(ensure(c->d_types, sizeof(int) * n, &c->alloc_generation));
    TRY(ensure(c->d_mol, sizeof(int) * n, &c->alloc_generation));
    if (n > 0) {
        HIP_TRY(hipMemcpy(c->d_types.p, t.data(), sizeof(int) * n, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->d_mol.p, m.data(), sizeof(int) * n, hipMemcpyHostToDevice));
    }
    if (c->has_excl) {
        TRY(ensure(c->d_excl_off, sizeof(int) * (n + 1), &c->alloc_generation));
        TRY(ensure(c->d_excl_idx, sizeof(int) * idx.size(), &c->alloc_generation));
        HIP_TRY(hipMemcpy(c->d_excl_off.p, off.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->d_excl_idx.p, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice));
    }
    c->topo_set = true;
    // bonded terms and the integrator describe the previous atoms
    c->has_bonded = false;
    c->md_ready = false;
    return RELRES_OK;
}

int relres_set_systems(relres_ctx* c, int nsys, const int* atom_offsets)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    if (!c->topo_set) return fail(RELRES_ERR_STATE, "relres_set_topology has not been called");
    if (nsys < 1 || !atom_offsets) return fail(RELRES_ERR_ARG, "need nsys >= 1 and atom_offsets");
    if (atom_offsets[0] != 0 || atom_offsets[nsys] != c->n)
        return fail(RELRES_ERR_ARG, "atom_offsets must run from 0 to n_atoms (%d)", c->n);
    std::vector<int> off(atom_offsets, atom_offsets + nsys + 1);
    std::vector<int> atoms(nsys), sites(nsys, 0), sys(c->n);
    for (int sy = 0; sy < nsys; ++sy) {
        if (off[sy + 1] < off[sy]) return fail(RELRES_ERR_ARG, "atom_offsets must not decrease");
        atoms[sy] = off[sy + 1] - off[sy];
        for (int i = off[sy]; i < off[sy + 1]; ++i) {
            sys[i] = sy;
            sites[sy] += c->hybrid[c->h_types[i]] ? 1 : 0;
        }
    }
    if (c->check_pending || c->status_in_graph) {
        TRY(fetch_status(c));
        c->nonfinite_seen = c->h_status->nonfinite;
        c->moved_seen = c->h_status->moved;
        c->check_pending = false;
    }
    c->ref_valid = false;
    c->warn_pending = false;
    if (nsys > 1 && c->n > 0) {
        TRY(ensure(c->d_sys, sizeof(int) * c->n, &c->alloc_generation));
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipMemcpy(c->d_sys.p, sys.data(), sizeof(int) * c->n, hipMemcpyHostToDevice));
    }
    c->nsys = nsys;
    c->skins.clear();                 // every system at the default skin
    c->sys_off = off;
    c->atoms_sys = atoms;
    c->sites_sys = sites;
    c->built = false;
    c->lanes_stale = true;
    if (nsys > 1) {
        // bonded terms and dynamics are single-system
        c->has_bonded = false;
        c->md_ready = false;
    }
    return RELRES_OK;
}

int relres_set_skins(relres_ctx* c, const double* skins)
{
    if (!c || !skins) return fail(RELRES_ERR_ARG, "NULL argument");
    if (!c->topo_set) return fail(RELRES_ERR_STATE, "relres_set_topology has not been called");
    for (int sy = 0; sy < c->nsys; ++sy)
        if (!(std::isfinite(skins[sy]) && skins[sy] >= 0.0))
            return fail(RELRES_ERR_CUTOFF_ORDER, "bad skin %g of system %d", skins[sy], sy);
    c->skins.assign(skins, skins + c->nsys);
    c->built = false;                 // the lists of the old skins are not kept
    return RELRES_OK;
}

int relres_build_lists(relres_ctx* c, const double* pos, const double* box, void* stream)
{
    TRY(build_checked(c, pos, box, (hipStream_t)stream));
    return take_warning(c);
}

int relres_build_lists_async(relres_ctx* c, const double* pos, const double* box, void* stream)
{
    hipStream_t s = (hipStream_t)stream;
    TRY(drain_check(c));
    if (c->lanes_stale) return build_checked(c, pos, box, s);   // first build / new grids
    TRY(enqueue_build(c, pos, box, s));
    return RELRES_OK;
}

int relres_check_lists(relres_ctx* c)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    TRY(examine_status(c));
    // the status copy just examined also shows force calls enqueued before
    // the build whose energy/virial wait gave up
    TRY(take_ew_failures(c));
    return take_warning(c);
}

int relres_sync(relres_ctx* c, void* stream)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &capture));
    if (capture != hipStreamCaptureStatusNone)
        return fail(RELRES_ERR_STATE, "relres_sync on a stream that is being captured");
    HIP_TRY(hipStreamSynchronize(s));
    // the status only accumulates: a newer copy serves a pending build check too
    HIP_TRY(hipMemcpy(c->h_status, c->d_status.p, sizeof(Status), hipMemcpyDeviceToHost));
    return take_ew_failures(c);
}

int relres_moved_atoms(relres_ctx* c, const double* pos, void* stream, int* count)
{
    if (!c || !count) return fail(RELRES_ERR_ARG, "NULL argument");
    if (c->check_pending) TRY(examine_status(c));
    if (!c->built || !c->ref_valid) return fail(RELRES_ERR_NO_LISTS, "no lists: call relres_build_lists first");
    if (c->n > 0 && !pos) return fail(RELRES_ERR_ARG, "pos is NULL");
    hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &capture));
    if (capture != hipStreamCaptureStatusNone)
        return fail(RELRES_ERR_STATE, "relres_moved_atoms waits for its result: not in a captured stream");
    *count = 0;
    if (c->n == 0) return RELRES_OK;
    char* st = (char*)c->d_status.p;
    static_assert(offsetof(Status, moved_query) % 8 == 0, "moved_query starts a 64-bit word");
    HIP_TRY(launch_clear_words((unsigned long long*)(st + offsetof(Status, moved_query)), 1, s));
    HIP_TRY(launch_moved(c->n, pos, topo_of(c), c->d_grids.as<GridDev>(), c->d_wpos.as<double4>(),
                         c->d_status.as<Status>(), s));
    HIP_TRY(hipMemcpyAsync(&c->h_query->moved_query, st + offsetof(Status, moved_query),
                           sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *count = (int)c->h_query->moved_query;
    return RELRES_OK;
}

int relres_set_launch(relres_ctx* c, int lanes_atom, int lanes_site)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    for (int v : {lanes_atom, lanes_site})
        if (v < 0 || v > 64 || (v & (v - 1)))
            return fail(RELRES_ERR_ARG, "lanes per row must be 0 (automatic) or a power of two <= 64");
    c->lanes_a = lanes_atom;
    c->lanes_b = lanes_site;
    return RELRES_OK;
}

int relres_set_list_launch(relres_ctx* c, int rows_atom, int rows_site, int cand_per_lane)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    for (int v : {rows_atom, rows_site})
        if (v < 0 || v > kRowsPerWave)
            return fail(RELRES_ERR_ARG, "rows per wave must be 0 (automatic) or 1..%d", kRowsPerWave);
    if (cand_per_lane != 0 && cand_per_lane != 2 && cand_per_lane != 4)
        return fail(RELRES_ERR_ARG, "candidates per lane must be 0 (automatic), 2 or 4");
    c->rows_a = rows_atom;
    c->rows_s = rows_site;
    c->cand = cand_per_lane;
    return RELRES_OK;
}

int relres_set_cells(relres_ctx* c, int div_atom, int div_site)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    for (int v : {div_atom, div_site})
        if (v < 0 || v > 2)
            return fail(RELRES_ERR_ARG, "cells per list radius must be 0 (automatic), 1 or 2");
    c->div_a = div_atom;
    c->div_s = div_site;
    return RELRES_OK;
}

int relres_autotune(relres_ctx* c, const double* pos, const double* box, void* stream, int reps,
                    relres_tune* out)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    if (!out) return fail(RELRES_ERR_ARG, "out is NULL");
    if (!box) return fail(RELRES_ERR_ARG, "box is NULL");
    if (c->n > 0 && !pos) return fail(RELRES_ERR_ARG, "pos is NULL");
    if (reps < 1 || reps > 1000) return fail(RELRES_ERR_ARG, "reps must be 1..1000");
    hipStream_t s = (hipStream_t)stream;
    hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &capture));
    if (capture != hipStreamCaptureStatusNone)
        return fail(RELRES_ERR_STATE, "relres_autotune cannot run on a capturing stream");
    std::memset(out, 0, sizeof *out);
    const bool sites = c->n_sites > 0;
    const bool was_timing = c->timing;
    TRY(relres_get_timing(c, nullptr, nullptr, nullptr, nullptr));   // start from empty tallies
    c->timing = true;
    int rc = RELRES_OK;
    DBuf f, e, w;
    long long gen = 0;
    // mean device time of `reps` timed builds (after one untimed) in us
    auto time_builds = [&](double& us) -> int {
        TRY(build_checked(c, pos, box, s));
        TRY(relres_get_timing(c, nullptr, nullptr, nullptr, nullptr));
        for (int r = 0; r < reps; ++r) TRY(build_checked(c, pos, box, s));
        double ms = 0.0;
        long long calls = 0;
        TRY(relres_get_timing(c, nullptr, nullptr, &ms, &calls));
        us = calls > 0 ? 1e3 * ms / (double)calls : 0.0;
        return RELRES_OK;
    };
    auto time_forces = [&](double& us) -> int {
        void* fp = f.p;
        TRY(relres_forces(c, pos, fp, e.as<double>(), w.as<double>(), s));
        TRY(relres_get_timing(c, nullptr, nullptr, nullptr, nullptr));
        for (int r = 0; r < reps; ++r) TRY(relres_forces(c, pos, fp, e.as<double>(), w.as<double>(), s));
        double ms = 0.0;
        long long calls = 0;
        TRY(relres_get_timing(c, &ms, &calls, nullptr, nullptr));
        us = calls > 0 ? 1e3 * ms / (double)calls : 0.0;
        return RELRES_OK;
    };
    auto run = [&]() -> int {
        if (c->n == 0) return RELRES_OK;
        // list kernel: rows per wave of each grid and candidates per lane;
        // the automatic choice first, as the reference point
        // and the cell size of each grid (one or half a list radius), grid
        // by grid outermost so the cell tables are rebuilt only when it changes
        struct ListShape { int da, ds, ra, rs, k; };
        std::vector<ListShape> shapes{{0, 0, 0, 0, 0}};
        for (int da : {1, 2})
            for (int ds : {1, 2}) {
                if (!sites && ds != da) continue;
                for (int k : {2, 4})
                    for (int ra : {4, 8, 16})
                        for (int rs : {4, 8, 16})
                            if (sites || rs == ra) shapes.push_back({da, ds, ra, rs, k});
            }
        double best = 0.0;
        ListShape pick{0, 0, 0, 0, 0};
        for (size_t i = 0; i < shapes.size(); ++i) {
            TRY(relres_set_cells(c, shapes[i].da, shapes[i].ds));
            TRY(relres_set_list_launch(c, shapes[i].ra, shapes[i].rs, shapes[i].k));
            double us = 0.0;
            TRY(time_builds(us));
            if (i == 0) out->build_us_auto = us;
            if (i == 0 || us < best) {
                best = us;
                pick = shapes[i];
            }
            out->trials++;
        }
        TRY(relres_set_cells(c, pick.da, pick.ds));
        TRY(relres_set_list_launch(c, pick.ra, pick.rs, pick.k));
        TRY(build_checked(c, pos, box, s));
        out->build_us = best;
        out->cell_div_atom = c->ga.div;
        out->cell_div_site = sites ? c->gs.div : 0;
        out->rows_atom = c->ga.rpw;
        out->rows_site = sites ? c->gs.rpw : 0;
        out->cand_per_lane = list_candidates(c->ga.waves + (sites ? c->gs.waves : 0), c->cand);
        // force kernel: lanes per atom row and per hybrid row
        const size_t fb = (size_t)c->n * 3 * (c->precision == 32 ? sizeof(float) : sizeof(double));
        TRY(ensure(f, fb, &gen));
        TRY(ensure(e, sizeof(double) * 3 * (size_t)c->nsys, &gen));
        TRY(ensure(w, sizeof(double) * 6 * (size_t)c->nsys, &gen));
        std::vector<std::pair<int, int>> lanes{{0, 0}};
        for (int la : {2, 4, 8, 16})
            for (int lb : {2, 4, 8, 16, 32})
                if (sites || lb == 16) lanes.push_back({la, lb});
        std::pair<int, int> lpick{0, 0};
        for (size_t i = 0; i < lanes.size(); ++i) {
            TRY(relres_set_launch(c, lanes[i].first, lanes[i].second));
            double us = 0.0;
            TRY(time_forces(us));
            if (i == 0) out->force_us_auto = us;
            if (i == 0 || us < best) {
                best = us;
                lpick = lanes[i];
            }
            out->trials++;
        }
        TRY(relres_set_launch(c, lpick.first, lpick.second));
        out->force_us = best;
        out->lanes_atom = lpick.first ? lpick.first : c->auto_la;
        out->lanes_site = lpick.second ? lpick.second : c->auto_lb;
        return RELRES_OK;
    };
    const int saved[7] = {c->rows_a, c->rows_s, c->cand, c->lanes_a, c->lanes_b, c->div_a,
                          c->div_s};
    rc = run();
    if (rc != RELRES_OK) {            // the caller's shapes again, not a trial's
        c->rows_a = saved[0];
        c->rows_s = saved[1];
        c->cand = saved[2];
        c->lanes_a = saved[3];
        c->lanes_b = saved[4];
        c->div_a = saved[5];
        c->div_s = saved[6];
    }
    const hipError_t sync = hipStreamSynchronize(s);   // temporaries are idle before release
    release(f);
    release(e);
    release(w);
    (void)relres_get_timing(c, nullptr, nullptr, nullptr, nullptr);
    c->timing = was_timing;
    if (rc == RELRES_OK && sync != hipSuccess)
        rc = fail(RELRES_ERR_HIP, "hipStreamSynchronize: %s", hipGetErrorString(sync));
    return rc;
}

namespace {

// Arguments of one force launch over the lists of the last build, with the
// lane split of the context; energy/virial buffers are the caller's.
ForceArgs force_args(const relres_ctx* c, const double* pos, void* forces, double* energy,
                     double* virial)
{
    const bool sites = c->n_sites > 0;
    const int la = c->lanes_a ? c->lanes_a : c->auto_la;
    const int lb = c->lanes_b ? c->lanes_b : c->auto_lb;
    auto blocks = [](long long rows, int lanes) {
        long long b = (rows * lanes + kForceBlock - 1) / kForceBlock;
        return (int)((b + 7) / 8 * 8);
    };
    ForceArgs a{};
    a.pos = pos;
    for (int k = 0; k < 3; ++k) {
        a.box[k] = c->box[k];
        a.inv_box[k] = 1.0 / c->box[k];
    }
    a.nsys = c->nsys;
    a.boxes = c->d_boxes.as<double>();
    a.n_arow = c->n;
    a.a_rec = c->d_a_rec.as<int4>();
    a.a_list = c->ga.list.as<int>();
    a.a_cap = c->ga.cap;
    a.n_srow = sites ? c->n_sites : 0;
    if (sites) {
        a.s_rec = c->d_s_rec.as<int4>();
        a.s_list = c->gs.list.as<int>();
        a.s_cap = c->gs.cap;
    }
    a.coef32 = c->d_coef32.p;
    a.coef64 = c->d_coef64.p;
    a.pcut32 = c->d_pcut32.as<Cutoffs<float>>();
    a.pcut64 = c->d_pcut64.as<Cutoffs<double>>();
    a.ntypes = c->ntypes;
    a.forces = forces;
    a.energy = energy;
    a.virial = virial;
    a.blocks_a = blocks(c->n, la);
    a.blocks_b = sites ? blocks(c->n_sites, lb) : 0;
    a.lanes_a = la;
    a.lanes_b = lb;
    a.log_lanes_a = log2i(la);
    a.log_lanes_b = log2i(lb);
    a.ew_failed = reinterpret_cast<unsigned int*>(static_cast<char*>(c->d_status.p) +
                                                  offsetof(Status, ew_failed));
    a.spin_limit = c->spin_limit;
    // rows of at least 8 list entries per lane (from the last list
    // statistics) take 4 entries per lane per batch in forces-only launches
    const double avg_a = c->n ? (double)c->stats.atom_entries / c->n : 0.0;
    const double avg_s = c->n_sites ? (double)c->stats.site_entries / c->n_sites : 0.0;
    a.wide_batch = c->n > 0 && avg_a >= 8.0 * la && (!sites || avg_a + avg_s >= 8.0 * lb);
    return a;
}

}  // namespace

int relres_forces(relres_ctx* c, const double* pos, void* forces, double* energy, double* virial,
                  void* stream)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    if (!c->built) return fail(RELRES_ERR_NO_LISTS, "no lists: call relres_build_lists first");
    hipStream_t s = (hipStream_t)stream;
    if (c->n == 0) {
        if (energy || virial) HIP_TRY(launch_zero_outputs(energy, virial, c->nsys, s));
        return RELRES_OK;
    }
    if (!pos || !forces) return fail(RELRES_ERR_ARG, "pos or forces is NULL");
    const bool sites = c->n_sites > 0;
    ForceArgs a = force_args(c, pos, forces, energy, virial);
    {
        // energy/virial records: a fresh buffer may hold another context's
        // records, whose tags could match this context's; clear it (tag 0)
        const long long g0 = c->alloc_generation;
        const size_t rec_bytes = (size_t)kEwRecBytes * (size_t)(a.blocks_a + a.blocks_b + kEwGroups);
        TRY(ensure(c->d_partials, rec_bytes, &c->alloc_generation));
        if (c->alloc_generation != g0)
            HIP_TRY(launch_clear_words(c->d_partials.as<unsigned long long>(),
                                       c->d_partials.bytes / sizeof(unsigned long long), s));
    }
    a.ew_rec = c->d_partials.as<unsigned long long>();
    a.epoch = c->d_epoch.as<unsigned int>();
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &capture));
    const bool timed = c->timing && capture == hipStreamCaptureStatusNone;
    if (timed) {
        TRY(take_events(c, e0, e1));
        HIP_TRY(hipEventRecord(e0, s));
    }
    const bool ew = energy || virial;
    if (ew && c->nsys > 1) {
        const size_t waves = (size_t)(a.blocks_a + a.blocks_b) * (kForceBlock / 64);
        TRY(ensure(c->d_row_ew, sizeof(double) * 8 * (size_t)(c->n + c->n_sites), &c->alloc_generation));
        TRY(ensure(c->d_wave_ew, sizeof(double) * 8 * waves, &c->alloc_generation));
        TRY(ensure(c->d_wave_sys, sizeof(int) * waves, &c->alloc_generation));
        a.row_ew = c->d_row_ew.as<double>();
        a.wave_ew = c->d_wave_ew.as<double>();
        a.wave_sys = c->d_wave_sys.as<int>();
    }
    HIP_TRY(launch_forces(a, c->cut64, c->per_pair, c->pair_math, c->precision, ew, s));
    if (timed) {
        HIP_TRY(hipEventRecord(e1, s));
        c->ev_force.push_back({e0, e1});
    }
    if (ew && c->nsys > 1)
        HIP_TRY(launch_reduce_sys_ew(c->d_grids.as<GridDev>(), sites ? 2 : 1, a, energy, virial, s));
    return RELRES_OK;
}

int relres_forces_noalloc(relres_ctx* c, const double* pos, void* forces, double* energy,
                          double* virial, void* stream)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    if (!c->built) return fail(RELRES_ERR_NO_LISTS, "no lists: call relres_build_lists first");
    hipStream_t s = (hipStream_t)stream;
    if (c->n == 0) {
        if (energy || virial) HIP_TRY(launch_zero_outputs(energy, virial, c->nsys, s));
        return RELRES_OK;
    }
    if (!pos || !forces) return fail(RELRES_ERR_ARG, "pos or forces is NULL");
    const bool ew = energy || virial;
    if (ew && c->nsys > 1)
        return fail(RELRES_ERR_ARG, "relres_forces_noalloc: energy/virial of several systems need "
                    "per-row buffers (use relres_forces, or pass NULL energy and virial)");
    if (!c->scratch)
        return fail(RELRES_ERR_HIP, "relres_forces_noalloc: no address for the static scratch "
                    "on device %d: %s", c->device, hipGetErrorString(c->scratch_err));
    ForceArgs a = force_args(c, pos, forces, energy, virial);
    const size_t need = kScratchEpochBytes +
                        (size_t)kEwRecBytes * (size_t)(a.blocks_a + a.blocks_b + kEwGroups);
    if (ew && need > kScratchBytes)
        return fail(RELRES_ERR_ARG, "relres_forces_noalloc: this launch needs %zu bytes of "
                    "energy/virial scratch, the static array holds %zu (fewer lanes per row "
                    "or relres_forces)", need, (size_t)kScratchBytes);
    // epoch first, records after it; records of earlier calls carry older
    // tags (the epoch only advances), so nothing needs clearing
    a.epoch = static_cast<unsigned int*>(c->scratch);
    a.ew_rec = reinterpret_cast<unsigned long long*>(static_cast<char*>(c->scratch) + kScratchEpochBytes);
    HIP_TRY(launch_forces(a, c->cut64, c->per_pair, c->pair_math, c->precision, ew, s));
    return RELRES_OK;
}

int relres_set_pair_params(relres_ctx* c, const double* eps_fg, const double* sig_fg,
                           const double* eps_cg, const double* sig_cg)
{
    if (!c || !eps_fg || !sig_fg || !eps_cg || !sig_cg) return fail(RELRES_ERR_ARG, "NULL argument");
    const int nt = c->ntypes;
    for (int a = 0; a < nt; ++a)
        for (int b = 0; b < nt; ++b) {
            const size_t q = (size_t)a * nt + b;
            if (!(std::isfinite(eps_fg[q]) && eps_fg[q] >= 0.0 && std::isfinite(sig_fg[q]) &&
                  sig_fg[q] > 0.0))
                return fail(RELRES_ERR_ARG, "bad FG pair parameters for types (%d, %d)", a, b);
            if (c->hybrid[a] && c->hybrid[b] &&
                !(std::isfinite(eps_cg[q]) && eps_cg[q] >= 0.0 && std::isfinite(sig_cg[q]) &&
                  sig_cg[q] > 0.0))
                return fail(RELRES_ERR_ARG, "bad CG pair parameters for types (%d, %d)", a, b);
        }
    // the tables may be in use by work still queued on any stream
    HIP_TRY(hipDeviceSynchronize());
    build_tables(c, eps_fg, sig_fg, eps_cg, sig_cg);
    c->tables_from_types = false;
    TRY(upload_tables(c));
    return RELRES_OK;
}

int relres_set_type_params(relres_ctx* c, const double* eps_fg, const double* sig_fg,
                           const double* eps_cg, const double* sig_cg)
{
    if (!c || !eps_fg || !sig_fg || !eps_cg || !sig_cg) return fail(RELRES_ERR_ARG, "NULL argument");
    const int nt = c->ntypes;
    for (int t = 0; t < nt; ++t) {
        if (!(std::isfinite(eps_fg[t]) && eps_fg[t] >= 0.0 && std::isfinite(sig_fg[t]) &&
              sig_fg[t] > 0.0))
            return fail(RELRES_ERR_ARG, "bad FG parameters for type %d", t);
        // the hybrid types define the site list: they may not change here
        if (c->hybrid[t] ? !(std::isfinite(eps_cg[t]) && eps_cg[t] > 0.0 &&
                             std::isfinite(sig_cg[t]) && sig_cg[t] > 0.0)
                         : eps_cg[t] != 0.0)
            return fail(RELRES_ERR_ARG, "type %d: eps_CG must stay %s (with sigma_CG > 0)", t,
                        c->hybrid[t] ? "positive" : "zero");
    }
    HIP_TRY(hipDeviceSynchronize());   // the tables may be in use by queued work
    std::vector<double> jac;
    install_type_params(c, eps_fg, sig_fg, eps_cg, sig_cg, jac);
    TRY(upload_tables(c));
    HIP_TRY(hipMemcpy(c->d_mix_jac.p, jac.data(), sizeof(double) * jac.size(), hipMemcpyHostToDevice));
    return RELRES_OK;
}

namespace {

int enqueue_backward(relres_ctx* c, const double* pos, const double* grad_forces,
                     const double* grad_energy, double* grad_pos, double* grad_pair, hipStream_t s);

}  // namespace

int relres_backward(relres_ctx* c, const double* pos, const double* grad_forces,
                    const double* grad_energy, double* grad_pos, double* grad_pair, void* stream)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    if (!grad_pair) return fail(RELRES_ERR_ARG, "grad_pair is NULL");
    return enqueue_backward(c, pos, grad_forces, grad_energy, grad_pos, grad_pair,
                            (hipStream_t)stream);
}

int relres_backward_types(relres_ctx* c, const double* pos, const double* grad_forces,
                          const double* grad_energy, double* grad_pos, double* grad_type,
                          void* stream)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    if (!grad_type) return fail(RELRES_ERR_ARG, "grad_type is NULL");
    if (!c->tables_from_types)
        return fail(RELRES_ERR_STATE, "pair parameters were set by relres_set_pair_params: "
                    "no per-type parameters to differentiate");
    const int nt = c->ntypes;
    for (int t = 0; t < nt; ++t) {
        const double* v = c->type_par.data();
        if (!(v[t] > 0.0 && v[nt + t] > 0.0) ||
            (c->hybrid[t] && !(v[2 * nt + t] > 0.0 && v[3 * nt + t] > 0.0)))
            return fail(RELRES_ERR_ARG, "type %d: per-type gradients need positive eps and sigma "
                        "(the mixing rules are not differentiable at zero)", t);
    }
    hipStream_t s = (hipStream_t)stream;
    TRY(enqueue_backward(c, pos, grad_forces, grad_energy, grad_pos, c->d_gpair.as<double>(), s));
    HIP_TRY(launch_type_grad(c->d_gpair.as<double>(), c->d_mix_jac.as<double>(), nt, grad_type, s));
    return RELRES_OK;
}

namespace {

int enqueue_backward(relres_ctx* c, const double* pos, const double* grad_forces,
                     const double* grad_energy, double* grad_pos, double* grad_pair, hipStream_t s)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    if (c->check_pending) TRY(examine_status(c));
    if (!c->built) return fail(RELRES_ERR_NO_LISTS, "no lists: call relres_build_lists first");
    if (c->ntypes > kBackwardTypes)
        return fail(RELRES_ERR_ARG, "relres_backward supports at most %d types (got %d)",
                    kBackwardTypes, c->ntypes);
    if (c->n > 0 && (!pos || !grad_pos)) return fail(RELRES_ERR_ARG, "pos or grad_pos is NULL");
    const int nt = c->ntypes;
    const int nbins = 4 * nt * nt;
    BackArgs b{};
    ForceArgs& a = b.f;
    const bool sites = c->n_sites > 0;
    const int la = c->lanes_a ? c->lanes_a : c->auto_la;
    const int lb = c->lanes_b ? c->lanes_b : c->auto_lb;
    auto blocks = [](long long rows, int lanes) {
        long long k = (rows * lanes + kForceBlock - 1) / kForceBlock;
        return (int)((k + 7) / 8 * 8);
    };
    a.pos = pos;
    for (int k = 0; k < 3; ++k) {
        a.box[k] = c->box[k];
        a.inv_box[k] = 1.0 / c->box[k];
    }
    a.nsys = c->nsys;
    a.boxes = c->d_boxes.as<double>();
    a.n_arow = c->n;
    a.a_rec = c->d_a_rec.as<int4>();
    a.a_list = c->ga.list.as<int>();
    a.a_cap = c->ga.cap;
    a.n_srow = sites ? c->n_sites : 0;
    if (sites) {
        a.s_rec = c->d_s_rec.as<int4>();
        a.s_list = c->gs.list.as<int>();
        a.s_cap = c->gs.cap;
    }
    a.coef64 = c->d_coef64.p;
    a.pcut64 = c->d_pcut64.as<Cutoffs<double>>();
    a.ntypes = nt;
    a.blocks_a = c->n > 0 ? blocks(c->n, la) : 0;
    a.blocks_b = (c->n > 0 && sites) ? blocks(c->n_sites, lb) : 0;
    a.lanes_a = la;
    a.lanes_b = lb;
    a.log_lanes_a = log2i(la);
    a.log_lanes_b = log2i(lb);
    b.gforce = grad_forces;
    b.genergy = grad_energy;
    b.gpos = grad_pos;
    b.cgrad = c->d_coef_grad.as<PairCoef<double>>();
    const int waves = (a.blocks_a + a.blocks_b) * (kForceBlock / 64);
    TRY(ensure(c->d_bpartial, sizeof(double) * (size_t)std::max(1, waves) * nbins, &c->alloc_generation));
    b.partial = c->d_bpartial.as<double>();
    HIP_TRY(launch_backward(b, waves, grad_pair, s));
    return RELRES_OK;
}

}  // namespace

int relres_set_bonded(relres_ctx* c, int nbonds, const int* bonds, const double* bond_k,
                      const double* bond_r0, int nangles, const int* angles, const double* angle_k,
                      const double* angle_t0, int ndihedrals, const int* dihedrals,
                      const double* dih_k, const int* dih_n, const double* dih_d, int npairs14,
                      const int* pairs14, double scale14)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    if (!c->topo_set) return fail(RELRES_ERR_STATE, "relres_set_topology has not been called");
    if (c->nsys != 1) return fail(RELRES_ERR_ARG, "bonded terms need a single system");
    const int n = c->n;
    if (nbonds < 0 || nangles < 0 || ndihedrals < 0 || npairs14 < 0)
        return fail(RELRES_ERR_ARG, "negative term count");
    if ((nbonds && (!bonds || !bond_k || !bond_r0)) ||
        (nangles && (!angles || !angle_k || !angle_t0)) ||
        (ndihedrals && (!dihedrals || !dih_k || !dih_n || !dih_d)) || (npairs14 && !pairs14))
        return fail(RELRES_ERR_ARG, "term array is NULL");
    if (!(std::isfinite(scale14) && scale14 >= 0.0)) return fail(RELRES_ERR_ARG, "bad 1-4 factor");
    const long long total = (long long)nbonds * 2 + (long long)nangles * 3 + (long long)ndihedrals * 4;
    if (std::max({nbonds, nangles, ndihedrals}) >= (1 << 28) || total > INT32_MAX)
        return fail(RELRES_ERR_ARG, "too many bonded terms");
    auto atom_ok = [n](int a) { return a >= 0 && a < n; };
    for (int t = 0; t < nbonds; ++t)
        if (!atom_ok(bonds[2 * t]) || !atom_ok(bonds[2 * t + 1]) || bonds[2 * t] == bonds[2 * t + 1] ||
            !(std::isfinite(bond_k[t]) && std::isfinite(bond_r0[t]) && bond_r0[t] > 0.0))
            return fail(RELRES_ERR_TOPOLOGY, "bad bond %d", t);
    for (int t = 0; t < nangles; ++t) {
        const int* q = angles + 3 * t;
        if (!atom_ok(q[0]) || !atom_ok(q[1]) || !atom_ok(q[2]) || q[0] == q[1] || q[1] == q[2] ||
            q[0] == q[2] || !(std::isfinite(angle_k[t]) && std::isfinite(angle_t0[t])))
            return fail(RELRES_ERR_TOPOLOGY, "bad angle %d", t);
    }
    for (int t = 0; t < ndihedrals; ++t) {
        const int* q = dihedrals + 4 * t;
        bool ok = std::isfinite(dih_k[t]) && std::isfinite(dih_d[t]) && dih_n[t] >= 0;
        for (int u = 0; u < 4; ++u) ok = ok && atom_ok(q[u]);
        for (int u = 0; u < 4 && ok; ++u)
            for (int v = u + 1; v < 4; ++v) ok = ok && q[u] != q[v];
        if (!ok) return fail(RELRES_ERR_TOPOLOGY, "bad dihedral %d", t);
    }
    for (int t = 0; t < npairs14; ++t)
        if (!atom_ok(pairs14[2 * t]) || !atom_ok(pairs14[2 * t + 1]) ||
            pairs14[2 * t] == pairs14[2 * t + 1])
            return fail(RELRES_ERR_TOPOLOGY, "bad 1-4 pair %d", t);

    // per atom: the terms it belongs to (bonds, angles, dihedrals, in order),
    // then its 1-4 partners (ascending)
    std::vector<std::vector<BondItem>> per(n);
    auto add = [&](int atom, int kind, int slot, int t, const int* q) {
        BondItem it{};
        it.kind = kind;
        it.slot = slot;
        it.i = q[0];
        it.j = q[1];
        it.k = kind >= 1 ? q[2] : 0;
        it.l = kind == 2 ? q[3] : 0;
        it.par = t;
        per[atom].push_back(it);
    };
    for (int t = 0; t < nbonds; ++t)
        for (int u = 0; u < 2; ++u) add(bonds[2 * t + u], 0, u, t, bonds + 2 * t);
    for (int t = 0; t < nangles; ++t)
        for (int u = 0; u < 3; ++u) add(angles[3 * t + u], 1, u, t, angles + 3 * t);
    for (int t = 0; t < ndihedrals; ++t)
        for (int u = 0; u < 4; ++u) add(dihedrals[4 * t + u], 2, u, t, dihedrals + 4 * t);
    std::vector<std::vector<int>> part(n);
    for (int t = 0; t < npairs14; ++t) {
        part[pairs14[2 * t]].push_back(pairs14[2 * t + 1]);
        part[pairs14[2 * t + 1]].push_back(pairs14[2 * t]);
    }
    const int nt = c->ntypes;
    for (int a = 0; a < n; ++a) {
        std::sort(part[a].begin(), part[a].end());
        for (int j : part[a]) {
            BondItem it{};
            it.kind = 3;
            it.i = a;
            it.j = j;
            it.par = c->h_types[a] * nt + c->h_types[j];
            per[a].push_back(it);
        }
    }
    // items per atom: a power of two holding every atom's list; lanes per
    // atom: as many, at most 32 (more items are taken in turns)
    size_t most = 1;
    for (int a = 0; a < n; ++a) most = std::max(most, per[a].size());
    if (most > 4096) return fail(RELRES_ERR_TOPOLOGY, "an atom has %zu bonded items (max 4096)", most);
    int slots = 1;
    while ((size_t)slots < most) slots <<= 1;
    int lg = 0;
    while ((1 << lg) < slots && lg < 5) ++lg;
    BondItem none{};
    none.kind = -1;
    std::vector<BondItem> items((size_t)n * slots, none);
    for (int a = 0; a < n; ++a)
        std::copy(per[a].begin(), per[a].end(), items.begin() + (size_t)a * slots);
    std::vector<double2> hbp(nbonds);
    for (int t = 0; t < nbonds; ++t) hbp[t] = make_double2(bond_k[t], bond_r0[t]);
    std::vector<double2> hap(nangles);
    for (int t = 0; t < nangles; ++t) hap[t] = make_double2(angle_k[t], angle_t0[t]);
    std::vector<double4> hdp(ndihedrals);
    for (int t = 0; t < ndihedrals; ++t)
        hdp[t] = make_double4(dih_k[t], (double)dih_n[t], std::cos(dih_d[t]), std::sin(dih_d[t]));
    // the buffers may be in use by work still queued on any stream
    HIP_TRY(hipDeviceSynchronize());
    long long* gen = &c->alloc_generation;
    auto up = [&](DBuf& b, const void* src, size_t bytes) -> int {
        TRY(ensure(b, bytes, gen));
        if (bytes) HIP_TRY(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
        return RELRES_OK;
    };
    TRY(up(c->d_items, items.data(), sizeof(BondItem) * items.size()));
    TRY(up(c->d_bond_par, hbp.data(), sizeof(double2) * hbp.size()));
    TRY(up(c->d_angle_par, hap.data(), sizeof(double2) * hap.size()));
    TRY(up(c->d_dih_par, hdp.data(), sizeof(double4) * hdp.size()));
    const int nblk = bonded_blocks(n, lg);
    TRY(ensure(c->d_bond_part, sizeof(double) * 10 * (size_t)std::max(1, nblk), gen));
    TRY(ensure(c->d_bond_sum, sizeof(double) * 16, gen));
    // kinetic partials of the kick (one per bonded block) and of k_md_kinetic
    TRY(ensure(c->d_md_part, sizeof(double) * (size_t)std::max({1, nblk, md_blocks(n)}), gen));
    c->bond_lg = lg;
    c->bond_slots = slots;
    c->scale14 = scale14;
    c->has_bonded = true;
    return RELRES_OK;
}

namespace {

int enqueue_bonded(relres_ctx* c, const double* pos, void* forces, bool sums, const MdArgs* m,
                   hipStream_t s)
{
    BondedArgs b{};
    b.pos = pos;
    for (int k = 0; k < 3; ++k) b.box[k] = c->box[k];
    b.n = c->n;
    b.items = c->d_items.as<BondItem>();
    b.slots = c->bond_slots;
    b.bond_par = c->d_bond_par.as<double2>();
    b.angle_par = c->d_angle_par.as<double2>();
    b.dih_par = c->d_dih_par.as<double4>();
    b.scale14 = c->scale14;
    b.coef64 = c->d_coef64.as<PairCoef<double>>();
    b.pcut64 = c->d_pcut64.as<Cutoffs<double>>();
    b.forces = forces;
    b.partial = sums ? c->d_bond_part.as<double>() : nullptr;
    b.log_lanes = c->bond_lg;
    HIP_TRY(launch_bonded(b, m, c->precision, s));
    if (sums)
        HIP_TRY(launch_sum_partials(c->d_bond_part.as<double>(), bonded_blocks(c->n, c->bond_lg),
                                    nullptr, 0, 10, c->d_bond_sum.as<double>(), s));
    return RELRES_OK;
}

}  // namespace

int relres_bonded_forces(relres_ctx* c, const double* pos, void* forces, double* energy,
                         double* virial, void* stream)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    if (!c->has_bonded) return fail(RELRES_ERR_STATE, "relres_set_bonded has not been called");
    if (!c->built) return fail(RELRES_ERR_NO_LISTS, "no box yet: call relres_build_lists first");
    if (c->n == 0) return RELRES_OK;
    if (!pos || !forces) return fail(RELRES_ERR_ARG, "pos or forces is NULL");
    hipStream_t s = (hipStream_t)stream;
    const bool sums = energy || virial;
    TRY(enqueue_bonded(c, pos, forces, sums, nullptr, s));
    const double* sum = c->d_bond_sum.as<double>();
    if (energy) HIP_TRY(hipMemcpyAsync(energy, sum, 4 * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (virial) HIP_TRY(hipMemcpyAsync(virial, sum + 4, 6 * sizeof(double), hipMemcpyDeviceToDevice, s));
    return RELRES_OK;
}

int relres_md_setup(relres_ctx* c, const double* masses, double dt, double kT, double tau,
                    double ftm2v, int rebuild_every)
{
    if (!c || !masses) return fail(RELRES_ERR_ARG, "NULL argument");
    if (!c->topo_set) return fail(RELRES_ERR_STATE, "relres_set_topology has not been called");
    if (c->nsys != 1) return fail(RELRES_ERR_ARG, "dynamics need a single system");
    if (!(dt > 0.0 && std::isfinite(dt) && kT > 0.0 && std::isfinite(kT) && tau > 0.0 &&
          ftm2v > 0.0 && std::isfinite(ftm2v) && rebuild_every >= 1 && c->n >= 2))
        return fail(RELRES_ERR_ARG, "need dt, kT, tau, ftm2v > 0, rebuild_every >= 1, n >= 2");
    const int n = c->n;
    for (int i = 0; i < n; ++i)
        if (!(masses[i] > 0.0 && std::isfinite(masses[i]))) return fail(RELRES_ERR_ARG, "bad mass %d", i);
    HIP_TRY(hipDeviceSynchronize());
    long long* gen = &c->alloc_generation;
    TRY(ensure(c->d_mass, sizeof(double) * n, gen));
    HIP_TRY(hipMemcpy(c->d_mass.p, masses, sizeof(double) * n, hipMemcpyHostToDevice));
    TRY(ensure(c->d_md_state, 2 * sizeof(MdState), gen));   // current and next
    TRY(ensure(c->d_md_xref, sizeof(double) * 3 * n, gen));
    TRY(ensure(c->d_md_F, (c->precision == 64 ? 8 : 4) * 3 * (size_t)n, gen));
    TRY(ensure(c->d_md_E, sizeof(double) * 3, gen));
    TRY(ensure(c->d_md_W, sizeof(double) * 6, gen));
    TRY(ensure(c->d_md_part, sizeof(double) * (size_t)std::max(md_blocks(n), bonded_blocks(n, c->bond_lg)), gen));
    TRY(ensure(c->d_md_stale, 64, gen));
    TRY(ensure(c->d_bond_sum, sizeof(double) * 16, gen));
    if (!c->h_stale && hipHostMalloc((void**)&c->h_stale, 64, hipHostMallocDefault) != hipSuccess)
        return fail(RELRES_ERR_HIP, "pinned host allocation failed");
    MdState st{};
    st.xi = st.eta = 0.0;
    st.K = 0.0;
    st.s2 = 1.0;
    st.s_apply = 1.0;
    st.s_last = 1.0;
    st.dt = dt;
    st.kT = kT;
    st.g = 3.0 * n - 3.0;
    st.Q = st.g * kT * tau * tau;
    HIP_TRY(hipMemcpy(c->d_md_state.p, &st, sizeof(MdState), hipMemcpyHostToDevice));
    c->md_cur = 0;
    c->md_ftm2v = ftm2v;
    c->md_rebuild = rebuild_every;
    // the per-atom bonded kernel also gives the half kick: without bonded
    // terms it runs with none
    if (!c->has_bonded)
        TRY(relres_set_bonded(c, 0, nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr, 0,
                              nullptr, nullptr, nullptr, nullptr, 0, nullptr, 0.0));
    c->md_ready = true;
    return RELRES_OK;
}

int relres_md_state(relres_ctx* c, double* xi, double* eta, int set)
{
    if (!c || !xi || !eta) return fail(RELRES_ERR_ARG, "NULL argument");
    if (!c->md_ready) return fail(RELRES_ERR_STATE, "relres_md_setup has not been called");
    HIP_TRY(hipDeviceSynchronize());
    MdState st{};
    MdState* cur = c->d_md_state.as<MdState>() + c->md_cur;
    HIP_TRY(hipMemcpy(&st, cur, sizeof(MdState), hipMemcpyDeviceToHost));
    if (set) {
        if (!(std::isfinite(*xi) && std::isfinite(*eta))) return fail(RELRES_ERR_ARG, "non-finite state");
        st.xi = *xi;
        st.eta = *eta;
        HIP_TRY(hipMemcpy(cur, &st, sizeof(MdState), hipMemcpyHostToDevice));
    } else {
        *xi = st.xi;
        *eta = st.eta;
    }
    return RELRES_OK;
}

namespace {

// Build the lists at pos (waiting for the build), after checking that no
// atom moved more than half the skin since the previous build.
int md_rebuild(relres_ctx* c, const double* pos, hipStream_t s, bool check)
{
    // the displacement flag of the steps since the previous build is copied
    // ahead of the build and read once the build has been waited for: one
    // host wait per rebuild, not two
    if (check)
        HIP_TRY(hipMemcpyAsync(c->h_stale, c->d_md_stale.p, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    const double box[3] = {c->box[0], c->box[1], c->box[2]};
    TRY(build_checked(c, pos, box, s));
    if (check && *c->h_stale)
        return fail(RELRES_ERR_STALE_LISTS, "an atom moved more than half the skin between list "
                    "builds: rebuild more often or use a larger skin");
    c->warn_pending = false;          // dynamics checks the displacements itself
    HIP_TRY(hipMemcpyAsync(c->d_md_xref.p, pos, sizeof(double) * 3 * c->n, hipMemcpyDeviceToDevice, s));
    HIP_TRY(launch_clear_words((unsigned long long*)c->d_md_stale.p, 8, s));
    return RELRES_OK;
}

}  // namespace

int relres_md_run(relres_ctx* c, double* pos, double* vel, int nsteps, int thermo_every,
                  double* thermo, void* stream)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    if (!c->md_ready) return fail(RELRES_ERR_STATE, "relres_md_setup has not been called");
    if (!c->built) return fail(RELRES_ERR_NO_LISTS, "no box yet: call relres_build_lists first");
    if (!pos || !vel || nsteps < 0 || thermo_every < 0 || (thermo_every > 0 && !thermo))
        return fail(RELRES_ERR_ARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    const int prec = c->precision;
    void* F = c->d_md_F.p;
    MdArgs m{};
    m.n = c->n;
    m.ftm2v = c->md_ftm2v;
    m.pos = pos;
    m.vel = vel;
    m.forces = F;
    m.mass = c->d_mass.as<double>();
    m.xref = c->d_md_xref.as<double>();
    m.half_skin2 = 0.25 * skin_of(c, 0) * skin_of(c, 0);
    m.stale = (unsigned*)c->d_md_stale.p;
    m.partial = c->d_md_part.as<double>();
    MdState* stb = c->d_md_state.as<MdState>();             // two buffers
    m.st = stb + c->md_cur;
    const int nblk = md_blocks(c->n);                       // partials of k_md_kinetic
    const int nblk_kick = bonded_blocks(c->n, c->bond_lg);  // partials of the kick
    const double* e_nb = c->d_md_E.as<double>();
    const double* w_nb = c->d_md_W.as<double>();
    const double* eb = c->d_bond_sum.as<double>();
    // forces at the starting positions, the kinetic energy and the first
    // thermostat half step
    TRY(md_rebuild(c, pos, s, false));
    TRY(relres_forces(c, pos, F, nullptr, nullptr, s));
    TRY(enqueue_bonded(c, pos, F, false, nullptr, s));
    HIP_TRY(launch_md_kinetic(m, s));
    HIP_TRY(launch_md_scalar(m.st, m.partial, nblk, m.ftm2v, 0, nsteps > 0, nullptr, nullptr,
                             nullptr, nullptr, s));
    auto row_of = [&](int step) -> double* {
        return thermo_every > 0 && step % thermo_every == 0
                   ? thermo + (size_t)8 * (step / thermo_every - 1) : nullptr;
    };
    for (int step = 1; step <= nsteps; ++step) {
        // from the second step on, the drift also does the scalar work after
        // the previous step (second thermostat half step, its row, first
        // half step of this one), reading one state buffer, writing the other
        if (step == 1) {
            HIP_TRY(launch_md_drift(m, m.st, m.st, 0, 0, nullptr, nullptr, nullptr, nullptr, prec, s));
        } else {
            const int next = 1 - c->md_cur;
            HIP_TRY(launch_md_drift(m, stb + c->md_cur, stb + next, nblk_kick, 1, e_nb, w_nb, eb,
                                    row_of(step - 1), prec, s));
            c->md_cur = next;
            m.st = stb + next;
        }
        if (step % c->md_rebuild == 0) TRY(md_rebuild(c, pos, s, true));
        const bool out = row_of(step) != nullptr;
        TRY(relres_forces(c, pos, F, out ? c->d_md_E.as<double>() : nullptr,
                          out ? c->d_md_W.as<double>() : nullptr, s));
        // bonded and 1-4 forces, the half kick and the kinetic partials
        TRY(enqueue_bonded(c, pos, F, out, &m, s));
    }
    // the second half step of the last step
    if (nsteps > 0)
        HIP_TRY(launch_md_scalar(m.st, m.partial, nblk_kick, m.ftm2v, 1, 0, e_nb, w_nb, eb,
                                 row_of(nsteps), s));
    HIP_TRY(launch_md_finish(m, s));
    // the last steps since the previous build must not have outrun the skin either
    HIP_TRY(hipMemcpyAsync(c->h_stale, c->d_md_stale.p, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (*c->h_stale)
        return fail(RELRES_ERR_STALE_LISTS, "an atom moved more than half the skin between list "
                    "builds: rebuild more often or use a larger skin");
    return RELRES_OK;
}

int relres_list_stats(relres_ctx* c, relres_stats* out)
{
    if (!c || !out) return fail(RELRES_ERR_ARG, "NULL argument");
    if (c->check_pending) TRY(examine_status(c));
    if (c->built && !c->stats_fresh) TRY(refresh_list_stats(c, nullptr));
    c->stats.atom_capacity = c->ga.cap;
    c->stats.site_capacity = c->n_sites > 0 ? c->gs.cap : 0;
    *out = c->stats;
    out->generation = c->alloc_generation;
    return RELRES_OK;
}

int relres_generation(relres_ctx* c, long long* generation)
{
    if (!c || !generation) return fail(RELRES_ERR_ARG, "NULL argument");
    *generation = c->alloc_generation;
    return RELRES_OK;
}

int relres_get_pairs(relres_ctx* c, int which, int* pairs_host, long long cap, long long* n_out)
{
    if (!c || !n_out) return fail(RELRES_ERR_ARG, "NULL argument");
    if (which != RELRES_LIST_ATOM && which != RELRES_LIST_SITE)
        return fail(RELRES_ERR_ARG, "which must be RELRES_LIST_ATOM or RELRES_LIST_SITE");
    if (cap > 0 && !pairs_host) return fail(RELRES_ERR_ARG, "pairs_host is NULL");
    if (c->check_pending) TRY(examine_status(c));
    if (!c->built) return fail(RELRES_ERR_NO_LISTS, "no lists");
    *n_out = 0;
    const bool site = which == RELRES_LIST_SITE;
    if (c->n == 0 || (site && c->n_sites == 0)) return RELRES_OK;
    GridHost& g = site ? c->gs : c->ga;
    const int rows = g.members;
    HIP_TRY(hipDeviceSynchronize());
    std::vector<int> nrow(rows), user(rows), list((size_t)rows * g.cap);
    HIP_TRY(hipMemcpy(nrow.data(), g.nrow.p, sizeof(int) * rows, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(user.data(), g.user.p, sizeof(int) * rows, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(list.data(), g.list.p, sizeof(int) * list.size(), hipMemcpyDeviceToHost));
    std::vector<std::pair<int, int>> pr;
    for (int r = 0; r < rows; ++r) {
        const int ui = user[r];
        const int cnt = std::min(nrow[r], g.cap);
        for (int k = 0; k < cnt; ++k) {
            const int uj = (int)((uint32_t)list[(size_t)r * g.cap + k] & kIdxMask);
            if (ui < uj) pr.push_back({ui, uj});
        }
    }
    std::sort(pr.begin(), pr.end());
    *n_out = (long long)pr.size();
    const long long w = std::min<long long>(cap, (long long)pr.size());
    for (long long k = 0; k < w; ++k) {
        pairs_host[2 * k] = pr[k].first;
        pairs_host[2 * k + 1] = pr[k].second;
    }
    return RELRES_OK;
}

int relres_set_timing(relres_ctx* c, int enable)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    c->timing = enable != 0;
    return RELRES_OK;
}

int relres_get_timing(relres_ctx* c, double* force_ms, long long* force_calls, double* build_ms,
                      long long* build_calls)
{
    if (!c) return fail(RELRES_ERR_ARG, "ctx is NULL");
    for (auto* v : {&c->ev_force, &c->ev_build}) {
        for (auto& pr : *v) {
            HIP_TRY(hipEventSynchronize(pr.second));
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
            if (v == &c->ev_force) { c->force_ms += ms; c->force_calls++; }
            else { c->build_ms += ms; c->build_calls++; }
            c->ev_free.push_back(pr.first);
            c->ev_free.push_back(pr.second);
        }
        v->clear();
    }
    if (force_ms) *force_ms = c->force_ms;
    if (force_calls) *force_calls = c->force_calls;
    if (build_ms) *build_ms = c->build_ms;
    if (build_calls) *build_calls = c->build_calls;
    c->force_ms = c->build_ms = 0.0;
    c->force_calls = c->build_calls = 0;
    return RELRES_OK;
}

void relres_destroy(relres_ctx* c)
{
    if (!c) return;
    (void)hipDeviceSynchronize();
    for (DBuf* b : {&c->d_coef_grad, &c->d_bpartial, &c->d_sys, &c->d_boxes, &c->d_row_ew, &c->d_wave_ew,
                    &c->d_wave_sys}) release(*b);
    for (DBuf* b : {&c->d_items, &c->d_bond_par, &c->d_angle_par, &c->d_dih_par,
                    &c->d_bond_part, &c->d_bond_sum,
                    &c->d_mass, &c->d_md_state, &c->d_md_xref,
                    &c->d_md_F, &c->d_md_E, &c->d_md_W, &c->d_md_part, &c->d_md_stale})
        release(*b);
    if (c->h_stale) (void)hipHostFree(c->h_stale);
    for (DBuf* b : {&c->d_coef64, &c->d_coef32, &c->d_hybrid, &c->d_types, &c->d_mol, &c->d_excl_off,
                    &c->d_excl_idx, &c->d_grids, &c->d_wpos, &c->d_key_a, &c->d_key_s,
                    &c->d_user2arow, &c->d_a_rec, &c->d_s_rec, &c->d_status, &c->d_partials, &c->d_seg_tot,
                    &c->d_epoch})
        release(*b);
    for (GridHost* g : {&c->ga, &c->gs})
        for (DBuf* b : {&g->geom_dev, &g->wave_sys_dev, &g->cell_sys, &g->rank_of_lin, &g->lin_of_rank, &g->nbr,
                        &g->count, &g->start, &g->user_unsorted, &g->user, &g->pos, &g->meta,
                        &g->row_cell, &g->list, &g->nrow})
            release(*b);
    if (c->h_grids) (void)hipHostFree(c->h_grids);
    if (c->h_status) (void)hipHostFree(c->h_status);
    if (c->h_query) (void)hipHostFree(c->h_query);
    for (auto* v : {&c->ev_force, &c->ev_build})
        for (auto& pr : *v) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (hipEvent_t e : c->ev_free) (void)hipEventDestroy(e);
    if (c->ev_status) (void)hipEventDestroy(c->ev_status);
    if (c->ev_upload) (void)hipEventDestroy(c->ev_upload);
    delete c;
}

}  // extern "C"

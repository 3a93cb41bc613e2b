/*
 * relres_oracle.c -- plain, slow, obviously correct FP64 reference for the
 * Relative Resolution (RelRes) Lennard-Jones pair computation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the package smoke check and the benchmark's
 * CPU-baseline leg do.  It shares no code, header, table or constant with the
 * HIP path.
 *
 * What it computes (paper: "Relative Resolution: A Computationally Efficient
 * Implementation in LAMMPS", arXiv:2104.10231):
 *   - per type pair: mixed FG/CG LJ parameters (Sec. 2.3, geometric mixing as
 *     stated there, Lorentz-Berthelot, or the sixth-power rule: the mixing
 *     rules the pair_modify mix keyword selects, Sec. 2.5), with the CG energy
 *     set to zero whenever a site is ordinary (Eq. 14);
 *   - per type pair: the four distances r_s-, r_s+, r_c-, r_c+ (Sec. 2.5: a
 *     global set, optionally overridden per type and mixed for unlike types
 *     with the same rule as sigma, as the geometric r_s of Sec. 3.4, or given
 *     per type pair outright);
 *   - the three smoothing polynomials of Eq. 16 obtained by SOLVING the
 *     boundary-condition systems of Eq. 7 (f_{s-}^{FG} at r_s-, f_{c-}^{CG} at
 *     r_c-) and Eq. 8 (f_{s+}^{CG} at r_s+) as 5x5 linear systems by Gaussian
 *     elimination; the closed forms of Eqs. 17/18 are deliberately NOT used
 *     here (the tests compare the two);
 *   - the shifting constants of Eq. 9, with the pair_modify shift option of
 *     Sec. 2.5 (shift no: Gamma_c- is zero where Eq. 20 subtracts it on its
 *     own, while Gamma_s+ and Gamma_s- keep their Eq. 9 values);
 *   - the pair potential of Eq. 20 evaluated directly, case by case;
 *   - the total energy of Eq. 3 as a sum over all non-excluded pairs i<j of a
 *     periodic orthorhombic box (minimum image), forces F_i = -dE/dx_i and the
 *     pair virial W_ab = sum_{i<j} d_a F_ij,b with d = x_i - x_j;
 *   - the two neighbour pair sets that a list-based code must find: atom pairs
 *     with r < r_s+ + skin and hybrid-hybrid pairs with r < r_c+ + skin;
 *   - the gradient of J = e_bar E + sum_i g_i . F_i with respect to the
 *     per-type parameters and the positions.  Every smoothing coefficient and
 *     shifting constant is a linear function of u, u', u'' at a zone
 *     boundary (Eqs. 7-9 are linear systems), so their parameter derivatives
 *     come from solving the same systems with differentiated right-hand
 *     sides; Eq. 20 is then differentiated case by case.
 *
 * Readings where the paper is silent or garbled:
 *   - Eq. 18 prints gamma_4+ with the wrong sign of its u'' term; the oracle
 *     does not use Eq. 18 at all, it solves Eq. 8 itself.
 *   - An empty smoothing zone (r_- == r_+, allowed in Sec. 2.5) makes the
 *     boundary system singular; the polynomial then reduces to its constant
 *     term, the potential value at the zone boundary.
 *   - Pair-set membership is decided in FP64 on wrapped positions:
 *       dx = x_j - x_i; if dx > L/2: dx -= L; else if dx < -L/2: dx += L;
 *       r2 = (dx*dx + dy*dy) + dz*dz;  member iff r2 < rl*rl, rl = r_+ + skin
 *     with every operation separately rounded (built with -ffp-contract=off).
 *   - Positions are wrapped into [0, L) by
 *       w = x - L*floor(x/L); if w < 0: w += L; if w >= L: w -= L;
 *       if w < 0 or w >= L: w = 0
 *   - An excluded pair loses both its FG and its CG part.
 *   - shift no: the paper states that the keyword acts on Gamma_c- alone and
 *     leaves Gamma_s+- untouched.  Read literally, cases 3 and 4 of Eq. 20
 *     subtract nothing, while cases 1 and 2 subtract Gamma_s- and Gamma_s+ as
 *     defined by Eq. 9 (which contain f_c-^CG(Dr_c)).  The potential then
 *     jumps by Gamma_c- at r_s+ and at r_c+; forces do not change.
 *   - Per-type distances of unlike types are mixed with the sigma rule
 *     (geometric, arithmetic or sixth-power mean of the two types' values),
 *     each of the four distances on its own; like types keep their own.
 *   - Sixth-power mixing: sigma_ab = ((sigma_a^6 + sigma_b^6)/2)^(1/6),
 *     eps_ab = 2 sqrt(eps_a eps_b) sigma_a^3 sigma_b^3 / (sigma_a^6 + sigma_b^6).
 *   - Neighbour pair sets use one radius per list: the largest r_s+ (atom
 *     list) or the largest hybrid-pair r_c+ (site list) plus the skin.
 *
 * Build: gcc -O2 -std=c99 -fPIC -shared -fopenmp -ffp-contract=off -lm
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Per-type-pair record, all FP64.  Layout (index: meaning):
 *   0 eps_fg  1 sig_fg  2 eps_cg  3 sig_cg
 *   4..8   gamma_{m-}^{FG} (m = 0..4), f_{s-}^{FG}, delta = r - r_s-
 *   9..13  gamma_{m+}^{CG} (m = 0..4), f_{s+}^{CG}, delta = r - r_s-
 *   14..18 gamma_{m-}^{CG} (m = 0..4), f_{c-}^{CG}, delta = r - r_c-
 *   19 Gamma_{c-} (Eq. 9)  20 Gamma_{s+}  21 Gamma_{s-}
 *   22..25 r_s-, r_s+, r_c-, r_c+ of this type pair
 *   26 the constant cases 3 and 4 of Eq. 20 subtract: Gamma_{c-}, or 0
 *      under shift no
 */
#define OR_REC 27
enum { R_EPS_FG = 0, R_SIG_FG, R_EPS_CG, R_SIG_CG, R_FG_SM = 4, R_CG_SP = 9,
       R_CG_CM = 14, R_G_CM = 19, R_G_SP = 20, R_G_SM = 21, R_CUT = 22, R_G_OUT = 26 };

int oracle_record_size(void) { return OR_REC; }

/* ---------------------------------------------------------------------------
 * LJ potential and its first two derivatives (Eqs. 11/12), textbook calculus:
 *   u   = 4 eps [ (s/r)^12 - (s/r)^6 ]
 *   u'  = 4 eps [ -12 s^12 / r^13 + 6 s^6 / r^7 ]
 *   u'' = 4 eps [ 156 s^12 / r^14 - 42 s^6 / r^8 ]
 * ------------------------------------------------------------------------- */
void oracle_lj(double eps, double sig, double r, double out[3])
{
    double q = sig / r;
    double q6 = q * q * q * q * q * q;
    double q12 = q6 * q6;
    out[0] = 4.0 * eps * (q12 - q6);
    out[1] = 4.0 * eps * (-12.0 * q12 + 6.0 * q6) / r;
    out[2] = 4.0 * eps * (156.0 * q12 - 42.0 * q6) / (r * r);
}

/* Row of the k-th derivative of sum_m gamma_m delta^m evaluated at delta. */
static void deriv_row(int k, double delta, double row[5])
{
    for (int m = 0; m < 5; ++m) {
        if (m < k) { row[m] = 0.0; continue; }
        double c = 1.0;
        for (int t = 0; t < k; ++t) c *= (double)(m - t);
        double p = 1.0;
        for (int t = 0; t < m - k; ++t) p *= delta;
        row[m] = c * p;
    }
}

/* Solve A x = b (5x5) by Gaussian elimination with partial pivoting. */
static int solve5(double A[5][5], double b[5], double x[5])
{
    for (int c = 0; c < 5; ++c) {
        int piv = c;
        for (int r = c + 1; r < 5; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (A[piv][c] == 0.0) return -1;
        if (piv != c) {
            for (int k = 0; k < 5; ++k) { double t = A[c][k]; A[c][k] = A[piv][k]; A[piv][k] = t; }
            double t = b[c]; b[c] = b[piv]; b[piv] = t;
        }
        for (int r = c + 1; r < 5; ++r) {
            double f = A[r][c] / A[c][c];
            for (int k = c; k < 5; ++k) A[r][k] -= f * A[c][k];
            b[r] -= f * b[c];
        }
    }
    for (int r = 4; r >= 0; --r) {
        double s = b[r];
        for (int k = r + 1; k < 5; ++k) s -= A[r][k] * x[k];
        x[r] = s / A[r][r];
    }
    return 0;
}

/* Smoothing polynomial coefficients from the boundary conditions.
 * kind 0 (switch-off, Eq. 7): f(0)=u, f'(0)=u', f''(0)=u'', f'(D)=0, f''(D)=0
 *                             with u = u(r_-)
 * kind 1 (switch-on,  Eq. 8): f(D)=u, f'(D)=u', f''(D)=u'', f'(0)=0, f''(0)=0
 *                             with u = u(r_+)
 * An empty zone (D == 0) keeps only the constant term f = u.              */
int oracle_solve_poly(int kind, double D, const double u[3], double gamma[5])
{
    if (D == 0.0) {
        gamma[0] = u[0];
        gamma[1] = gamma[2] = gamma[3] = gamma[4] = 0.0;
        return 0;
    }
    double A[5][5], b[5];
    double at_u = kind == 0 ? 0.0 : D;     /* where f matches u, u', u'' */
    double at_0 = kind == 0 ? D : 0.0;     /* where f', f'' vanish      */
    deriv_row(0, at_u, A[0]); b[0] = u[0];
    deriv_row(1, at_u, A[1]); b[1] = u[1];
    deriv_row(2, at_u, A[2]); b[2] = u[2];
    deriv_row(1, at_0, A[3]); b[3] = 0.0;
    deriv_row(2, at_0, A[4]); b[4] = 0.0;
    return solve5(A, b, gamma);
}

static double poly(const double g[5], double d)
{
    return g[0] + g[1] * d + g[2] * d * d + g[3] * d * d * d + g[4] * d * d * d * d;
}

static double dpoly(const double g[5], double d)
{
    return g[1] + 2.0 * g[2] * d + 3.0 * g[3] * d * d + 4.0 * g[4] * d * d * d;
}

/* Mixing rules (Sec. 2.3; Sec. 2.5 mix keyword).  mix: 0 geometric (eps and
 * sigma geometric means), 1 Lorentz-Berthelot (eps geometric, sigma
 * arithmetic), 2 sixth-power (see the readings above).                     */
static double mix_sigma(int mix, double a, double b)
{
    if (mix == 1) return 0.5 * (a + b);
    if (mix == 2) return pow(0.5 * (pow(a, 6.0) + pow(b, 6.0)), 1.0 / 6.0);
    return sqrt(a * b);
}

static double mix_eps(int mix, double ea, double eb, double sa, double sb)
{
    if (mix == 2) {
        double sa3 = sa * sa * sa, sb3 = sb * sb * sb;
        return 2.0 * sqrt(ea * eb) * sa3 * sb3 / (sa3 * sa3 + sb3 * sb3);
    }
    return sqrt(ea * eb);
}

/* Build the per-type-pair table (ntypes*ntypes records of OR_REC doubles).
 * A type is hybrid iff its CG energy parameter is positive; ordinary-involving
 * pairs get eps_CG = 0 (Eq. 14).  Distances of a pair: cut_pair[(a*ntypes +
 * b)*4 + k] if cut_pair is given, else cut_type[a*4 + k] for like types and
 * their mix for unlike ones if cut_type is given, else cut[k] (k = 0..3:
 * r_s-, r_s+, r_c-, r_c+).  shift = 0 selects pair_modify shift no.
 * Returns 0, or -1 when a pair violates r_s- <= r_s+ <= r_c- <= r_c+, -2 on
 * a singular solve.                                                          */
int oracle_setup(int ntypes, const double *eps_fg, const double *sig_fg,
                 const double *eps_cg, const double *sig_cg, int mix,
                 const double cut[4], const double *cut_type, const double *cut_pair,
                 int shift, double *table)
{
    for (int a = 0; a < ntypes; ++a)
        for (int b = 0; b < ntypes; ++b) {
            double *R = table + (size_t)(a * ntypes + b) * OR_REC;
            memset(R, 0, sizeof(double) * OR_REC);
            for (int k = 0; k < 4; ++k) {
                if (cut_pair) R[R_CUT + k] = cut_pair[(a * ntypes + b) * 4 + k];
                else if (cut_type && a == b) R[R_CUT + k] = cut_type[a * 4 + k];
                else if (cut_type) R[R_CUT + k] = mix_sigma(mix, cut_type[a * 4 + k], cut_type[b * 4 + k]);
                else R[R_CUT + k] = cut[k];
            }
            double rsi = R[R_CUT], rso = R[R_CUT + 1], rci = R[R_CUT + 2], rco = R[R_CUT + 3];
            if (!(0.0 <= rsi && rsi <= rso && rso <= rci && rci <= rco)) return -1;
            double Ds = rso - rsi, Dc = rco - rci;
            R[R_EPS_FG] = mix_eps(mix, eps_fg[a], eps_fg[b], sig_fg[a], sig_fg[b]);
            R[R_SIG_FG] = mix_sigma(mix, sig_fg[a], sig_fg[b]);
            int hybrid_pair = eps_cg[a] > 0.0 && eps_cg[b] > 0.0;
            R[R_EPS_CG] = hybrid_pair ? mix_eps(mix, eps_cg[a], eps_cg[b], sig_cg[a], sig_cg[b]) : 0.0;
            R[R_SIG_CG] = hybrid_pair ? mix_sigma(mix, sig_cg[a], sig_cg[b]) : 0.0;
            double u[3];
            /* f_{s-}^{FG}: switch-off of the FG potential, Eq. 7 at r_s- */
            oracle_lj(R[R_EPS_FG], R[R_SIG_FG], rsi, u);
            if (oracle_solve_poly(0, Ds, u, R + R_FG_SM)) return -2;
            if (hybrid_pair) {
                /* f_{s+}^{CG}: switch-on of the CG potential, Eq. 8 at r_s+ */
                oracle_lj(R[R_EPS_CG], R[R_SIG_CG], rso, u);
                if (oracle_solve_poly(1, Ds, u, R + R_CG_SP)) return -2;
                /* f_{c-}^{CG}: switch-off of the CG potential, Eq. 7 at r_c- */
                oracle_lj(R[R_EPS_CG], R[R_SIG_CG], rci, u);
                if (oracle_solve_poly(0, Dc, u, R + R_CG_CM)) return -2;
            }
            /* Eq. 9 */
            R[R_G_CM] = poly(R + R_CG_CM, Dc);
            R[R_G_SP] = poly(R + R_CG_CM, Dc) + poly(R + R_FG_SM, Ds);
            R[R_G_SM] = poly(R + R_CG_CM, Dc) + poly(R + R_FG_SM, Ds) - poly(R + R_CG_SP, 0.0);
            R[R_G_OUT] = shift ? R[R_G_CM] : 0.0;
        }
    return 0;
}

/* Eq. 20, case by case, with the record's own distances: returns u~(r),
 * stores du~/dr and the case index (1..5) that applied.                    */
double oracle_pair(const double *R, double r, double *dudr, int *which)
{
    const double *C = R + R_CUT;
    double rsi = C[0], rso = C[1], rci = C[2], rco = C[3];
    double u[3];
    if (r < rsi) {                                  /* [0, r_s-)     */
        oracle_lj(R[R_EPS_FG], R[R_SIG_FG], r, u);
        if (which) *which = 1;
        *dudr = u[1];
        return u[0] - R[R_G_SM];
    }
    if (r < rso) {                                  /* [r_s-, r_s+)  */
        double g[5], d = r - rsi;
        for (int m = 0; m < 5; ++m) g[m] = R[R_FG_SM + m] + R[R_CG_SP + m];
        if (which) *which = 2;
        *dudr = dpoly(g, d);
        return poly(g, d) - R[R_G_SP];
    }
    if (r < rci) {                                  /* [r_s+, r_c-)  */
        oracle_lj(R[R_EPS_CG], R[R_SIG_CG], r, u);
        if (which) *which = 3;
        *dudr = u[1];
        return u[0] - R[R_G_OUT];
    }
    if (r < rco) {                                  /* [r_c-, r_c+)  */
        double d = r - rci;
        if (which) *which = 4;
        *dudr = dpoly(R + R_CG_CM, d);
        return poly(R + R_CG_CM, d) - R[R_G_OUT];
    }
    if (which) *which = 5;                          /* [r_c+, inf)   */
    *dudr = 0.0;
    return 0.0;
}

/* Diagnostic split of Eq. 20 into the part carried by the FG potential and
 * the part carried by the CG potential (their sum is Eq. 20; used only to
 * report the FG/CG energy breakdown).                                       */
static void pair_split(const double *R, double r, double *e_fg, double *e_cg)
{
    const double *C = R + R_CUT;
    double rsi = C[0], rso = C[1], rci = C[2], rco = C[3];
    double Ds = rso - rsi, u[3];
    double fs_end = poly(R + R_FG_SM, Ds);
    if (r < rsi) { oracle_lj(R[R_EPS_FG], R[R_SIG_FG], r, u); *e_fg = u[0] - fs_end; }
    else if (r < rso) *e_fg = poly(R + R_FG_SM, r - rsi) - fs_end;
    else *e_fg = 0.0;
    if (r < rsi) *e_cg = R[R_CG_SP] - R[R_G_CM];
    else if (r < rso) *e_cg = poly(R + R_CG_SP, r - rsi) - R[R_G_CM];
    else if (r < rci) { oracle_lj(R[R_EPS_CG], R[R_SIG_CG], r, u); *e_cg = u[0] - R[R_G_OUT]; }
    else if (r < rco) *e_cg = poly(R + R_CG_CM, r - rci) - R[R_G_OUT];
    else *e_cg = 0.0;
}

/* ---------------------------------------------------------------------------
 * Periodic geometry
 * ------------------------------------------------------------------------- */
static double wrap1(double x, double L)
{
    double w = x - L * floor(x / L);
    if (w < 0.0) w += L;
    if (w >= L) w -= L;
    if (w < 0.0 || w >= L) w = 0.0;
    return w;
}

void oracle_wrap(int n, const double *pos, const double *box, double *out)
{
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 3; ++k) out[3 * i + k] = wrap1(pos[3 * i + k], box[k]);
}

/* d = x_j - x_i with the single-shift minimum image, on wrapped positions */
static void min_image(const double *xi, const double *xj, const double *box, double d[3])
{
    for (int k = 0; k < 3; ++k) {
        double dx = xj[k] - xi[k];
        double h = 0.5 * box[k];
        if (dx > h) dx -= box[k];
        else if (dx < -h) dx += box[k];
        d[k] = dx;
    }
}

static int is_excluded(int i, int j, const int *mol, int same_mol,
                       const int *eoff, const int *eidx)
{
    if (same_mol && mol[i] == mol[j]) return 1;
    if (eoff) {
        for (int k = eoff[i]; k < eoff[i + 1]; ++k) if (eidx[k] == j) return 1;
        for (int k = eoff[j]; k < eoff[j + 1]; ++k) if (eidx[k] == i) return 1;
    }
    return 0;
}

/* Energy (Eq. 3), forces and pair virial by brute force over all pairs.
 * Each atom i sums over every j != i (so no two threads write one atom);
 * E and W take each unordered pair once (j > i).  Per-atom partial sums are
 * combined serially in atom order, so results do not depend on the thread
 * count.  E_out = {E_total, E_FG part, E_CG part}; W_out = {xx,yy,zz,xy,xz,yz}.
 * If `sel` is non-NULL only the forces of atoms sel[0..nsel) are computed
 * (written to F rows 0..nsel) and E, W are not touched.                    */
int oracle_compute(int n, const double *pos, const double *box, const int *types,
                   const int *mol, int same_mol, const int *eoff, const int *eidx,
                   int ntypes, const double *table,
                   int nthreads, int nsel, const int *sel,
                   double *F, double *E_out, double *W_out)
{
    double *w = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    int nrows = sel ? nsel : n;
    double *pe = (double *)calloc((size_t)(nrows > 0 ? nrows : 1) * 9, sizeof(double));
    if (!w || !pe) { free(w); free(pe); return -1; }
    oracle_wrap(n, pos, box, w);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 16)
    for (int row = 0; row < nrows; ++row) {
        int i = sel ? sel[row] : row;
        double fx = 0.0, fy = 0.0, fz = 0.0;
        double *acc = pe + (size_t)row * 9;   /* E, Efg, Ecg, W[6] for j > i */
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            if (is_excluded(i, j, mol, same_mol, eoff, eidx)) continue;
            double d[3];
            min_image(w + 3 * i, w + 3 * j, box, d);   /* d = x_j - x_i */
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            const double *R = table + (size_t)(types[i] * ntypes + types[j]) * OR_REC;
            if (!(r < R[R_CUT + 3])) continue;         /* case 5: nothing */
            double dudr;
            double e = oracle_pair(R, r, &dudr, NULL);
            /* F_i = -dE/dx_i = -u~'(r) (x_i - x_j)/r = +u~'(r) d / r */
            double s = dudr / r;
            fx += s * d[0]; fy += s * d[1]; fz += s * d[2];
            if (j > i) {
                double efg, ecg;
                pair_split(R, r, &efg, &ecg);
                acc[0] += e; acc[1] += efg; acc[2] += ecg;
                /* W_ab += (x_i - x_j)_a F_ij,b with F_ij = +u~' d / r */
                double ra[3] = { -d[0], -d[1], -d[2] };
                double f[3] = { s * d[0], s * d[1], s * d[2] };
                acc[3] += ra[0] * f[0]; acc[4] += ra[1] * f[1]; acc[5] += ra[2] * f[2];
                acc[6] += ra[0] * f[1]; acc[7] += ra[0] * f[2]; acc[8] += ra[1] * f[2];
            }
        }
        F[3 * row + 0] = fx; F[3 * row + 1] = fy; F[3 * row + 2] = fz;
    }
    if (!sel) {
        double t[9] = {0};
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < 9; ++k) t[k] += pe[(size_t)i * 9 + k];
        for (int k = 0; k < 3; ++k) E_out[k] = t[k];
        for (int k = 0; k < 6; ++k) W_out[k] = t[3 + k];
    }
    free(w); free(pe);
    return 0;
}

/* Pair sets.  which = 0: all non-excluded pairs with r2 < (r_out + skin)^2;
 * which = 1: non-excluded hybrid-hybrid pairs with r2 < (r_out + skin)^2
 * (r_out: the largest r_s+, or the largest hybrid-pair r_c+).
 * Hybrid <=> hybrid_flag[type] != 0.  Pairs are written as (i, j) with i < j,
 * i-major then j ascending, up to `cap` pairs; the return value is the total
 * number of pairs (which may exceed cap).  If `row_sel` is non-NULL, only
 * rows i in row_sel[0..nrow) are enumerated, and j runs over ALL atoms
 * (ordered pairs (i, j), j != i), which gives full rows for sampled atoms. */
long oracle_pairs(int n, const double *pos, const double *box, const int *types,
                  const int *hybrid_flag, const int *mol, int same_mol,
                  const int *eoff, const int *eidx, double r_out, double skin,
                  int which, int nrow, const int *row_sel, int *out, long cap)
{
    double *w = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!w) return -1;
    oracle_wrap(n, pos, box, w);
    double rl = r_out + skin;
    double rl2 = rl * rl;
    long cnt = 0;
    int nr = row_sel ? nrow : n;
    for (int row = 0; row < nr; ++row) {
        int i = row_sel ? row_sel[row] : row;
        if (which == 1 && !hybrid_flag[types[i]]) continue;
        for (int j = row_sel ? 0 : i + 1; j < n; ++j) {
            if (j == i) continue;
            if (which == 1 && !hybrid_flag[types[j]]) continue;
            if (is_excluded(i, j, mol, same_mol, eoff, eidx)) continue;
            double d[3];
            min_image(w + 3 * i, w + 3 * j, box, d);
            double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
            if (r2 < rl2) {
                if (cnt < cap) { out[2 * cnt] = i; out[2 * cnt + 1] = j; }
                ++cnt;
            }
        }
    }
    free(w);
    return cnt;
}

/* Scaled 1-4 pairs (Sec. 3.2: the non-bonded interaction of atoms three bonds
 * apart is scaled down, by a factor 2 in the paper): Eq. 20 of each listed
 * pair (i, j) times `scale`, with d = x_j - x_i by the single-shift minimum
 * image.  Forces are ADDED to F; E_out = {total, FG part, CG part} and W_out
 * are added to.                                                            */
void oracle_pairs14(const double *pos, const double *box, const int *types, int ntypes,
                    const double *table, int np, const int *pairs, double scale,
                    double *F, double *E_out, double *W_out)
{
    for (int t = 0; t < np; ++t) {
        int i = pairs[2 * t], j = pairs[2 * t + 1];
        double d[3];
        min_image(pos + 3 * i, pos + 3 * j, box, d);        /* d = x_j - x_i */
        double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double *R = table + (size_t)(types[i] * ntypes + types[j]) * OR_REC;
        double dudr, efg, ecg;
        double u = oracle_pair(R, r, &dudr, NULL);
        pair_split(R, r, &efg, &ecg);
        double s = scale * dudr / r;                      /* F_i = +u~' d / r */
        double f[3] = {s * d[0], s * d[1], s * d[2]};
        for (int c = 0; c < 3; ++c) {
            F[3 * i + c] += f[c];
            F[3 * j + c] -= f[c];
        }
        E_out[0] += scale * u;
        E_out[1] += scale * efg;
        E_out[2] += scale * ecg;
        /* W += (x_i - x_j) (x) F_i */
        W_out[0] += -d[0] * f[0]; W_out[1] += -d[1] * f[1]; W_out[2] += -d[2] * f[2];
        W_out[3] += -d[0] * f[1]; W_out[4] += -d[0] * f[2]; W_out[5] += -d[1] * f[2];
    }
}

/* Evaluate Eq. 20 for a vector of distances with one type-pair record. */
void oracle_pair_vec(const double *R, int m, const double *r,
                     double *u, double *dudr, int *which, double *e_fg, double *e_cg)
{
    for (int k = 0; k < m; ++k) {
        u[k] = oracle_pair(R, r[k], dudr + k, which ? which + k : NULL);
        if (e_fg && e_cg) pair_split(R, r[k], e_fg + k, e_cg + k);
    }
}

/* ---------------------------------------------------------------------------
 * Gradients
 * ------------------------------------------------------------------------- */

/* Parameter derivative of u, u', u'' (Eqs. 11/12): wrt = 0 -> d/d eps,
 * wrt = 1 -> d/d sigma.  With q = sigma/r:
 *   du/deps   = 4 (q^12 - q^6)              du/dsig   = 4 eps (12 q^12 - 6 q^6) / sigma
 *   du'/deps  = 4 (-12 q^12 + 6 q^6) / r    du'/dsig  = 4 eps (-144 q^12 + 36 q^6) / (sigma r)
 *   du''/deps = 4 (156 q^12 - 42 q^6) / r^2 du''/dsig = 4 eps (1872 q^12 - 252 q^6) / (sigma r^2) */
static void lj_dparam(double eps, double sig, double r, int wrt, double out[3])
{
    double q = sig / r;
    double q6 = q * q * q * q * q * q;
    double q12 = q6 * q6;
    if (wrt == 0) {
        out[0] = 4.0 * (q12 - q6);
        out[1] = 4.0 * (-12.0 * q12 + 6.0 * q6) / r;
        out[2] = 4.0 * (156.0 * q12 - 42.0 * q6) / (r * r);
    } else {
        out[0] = 4.0 * eps * (12.0 * q12 - 6.0 * q6) / sig;
        out[1] = 4.0 * eps * (-144.0 * q12 + 36.0 * q6) / (sig * r);
        out[2] = 4.0 * eps * (1872.0 * q12 - 252.0 * q6) / (sig * r * r);
    }
}

static double d2poly(const double g[5], double d)
{
    return 2.0 * g[2] + 6.0 * g[3] * d + 12.0 * g[4] * d * d;
}

/* Derivative of a type-pair record with respect to one pair parameter
 * (P: 0 eps_FG, 1 sigma_FG, 2 eps_CG, 3 sigma_CG): the polynomial
 * coefficients solved from Eqs. 7/8 with the differentiated boundary values,
 * and Eq. 9 applied to them.  The CG part of a pair that is not hybrid-hybrid
 * is zero by Eq. 14 and does not depend on the CG parameters.              */
static int dparam_record(const double *R, int P, int shift, double *dR)
{
    const double *C = R + R_CUT;
    double rsi = C[0], rso = C[1], rci = C[2], rco = C[3];
    double Ds = rso - rsi, Dc = rco - rci, du[3];
    memset(dR, 0, sizeof(double) * OR_REC);
    if (P < 2) {
        lj_dparam(R[R_EPS_FG], R[R_SIG_FG], rsi, P, du);
        if (oracle_solve_poly(0, Ds, du, dR + R_FG_SM)) return -2;
    } else if (R[R_EPS_CG] > 0.0) {
        lj_dparam(R[R_EPS_CG], R[R_SIG_CG], rso, P - 2, du);
        if (oracle_solve_poly(1, Ds, du, dR + R_CG_SP)) return -2;
        lj_dparam(R[R_EPS_CG], R[R_SIG_CG], rci, P - 2, du);
        if (oracle_solve_poly(0, Dc, du, dR + R_CG_CM)) return -2;
    }
    dR[R_G_CM] = poly(dR + R_CG_CM, Dc);
    dR[R_G_SP] = poly(dR + R_CG_CM, Dc) + poly(dR + R_FG_SM, Ds);
    dR[R_G_SM] = poly(dR + R_CG_CM, Dc) + poly(dR + R_FG_SM, Ds) - poly(dR + R_CG_SP, 0.0);
    dR[R_G_OUT] = shift ? dR[R_G_CM] : 0.0;
    return 0;
}

/* d u~/dP and d u~'/dP at r: Eq. 20 differentiated case by case.           */
static void pair_dparam(const double *R, const double *dR, int P, double r,
                        double *du, double *dup)
{
    const double *C = R + R_CUT;
    double rsi = C[0], rso = C[1], rci = C[2], rco = C[3], v[3];
    if (r < rsi) {
        if (P < 2) {
            lj_dparam(R[R_EPS_FG], R[R_SIG_FG], r, P, v);
            *du = v[0] - dR[R_G_SM];
            *dup = v[1];
        } else {
            *du = -dR[R_G_SM];
            *dup = 0.0;
        }
    } else if (r < rso) {
        double g[5], d = r - rsi;
        for (int m = 0; m < 5; ++m) g[m] = dR[R_FG_SM + m] + dR[R_CG_SP + m];
        *du = poly(g, d) - dR[R_G_SP];
        *dup = dpoly(g, d);
    } else if (r < rci) {
        if (P >= 2 && R[R_EPS_CG] > 0.0) {
            lj_dparam(R[R_EPS_CG], R[R_SIG_CG], r, P - 2, v);
            *du = v[0] - dR[R_G_OUT];
            *dup = v[1];
        } else {
            *du = -dR[R_G_OUT];
            *dup = 0.0;
        }
    } else if (r < rco) {
        double d = r - rci;
        *du = poly(dR + R_CG_CM, d) - dR[R_G_OUT];
        *dup = dpoly(dR + R_CG_CM, d);
    } else {
        *du = 0.0;
        *dup = 0.0;
    }
}

/* Second derivative of Eq. 20, case by case. */
static double pair_d2(const double *R, double r)
{
    const double *C = R + R_CUT;
    double rsi = C[0], rso = C[1], rci = C[2], rco = C[3], u[3];
    if (r < rsi) { oracle_lj(R[R_EPS_FG], R[R_SIG_FG], r, u); return u[2]; }
    if (r < rso) {
        double g[5];
        for (int m = 0; m < 5; ++m) g[m] = R[R_FG_SM + m] + R[R_CG_SP + m];
        return d2poly(g, r - rsi);
    }
    if (r < rci) { oracle_lj(R[R_EPS_CG], R[R_SIG_CG], r, u); return u[2]; }
    if (r < rco) return d2poly(R + R_CG_CM, r - rci);
    return 0.0;
}

/* Partial derivatives of a mixed pair (eps_ab, sigma_ab) with respect to
 * the per-type values of type a (J[0] = d/d eps_a, J[1] = d/d sigma_a):
 *   geometric:    eps_ab = sqrt(ea eb), sigma_ab = sqrt(sa sb)
 *   Lorentz-Berthelot: sigma_ab = (sa + sb)/2
 *   sixth-power:  d eps_ab/d eps_a = eps_ab/(2 ea),
 *                 d eps_ab/d sa = eps_ab (3/sa - 6 sa^5/(sa^6 + sb^6)),
 *                 d sigma_ab/d sa = sa^5 / (2 sigma_ab^5).
 * de[] holds the eps_ab derivatives, ds[] the sigma_ab ones.  The values of
 * type b follow by swapping the arguments.                                */
static void mix_jacobian(int mix, double ea, double eb, double sa, double sb,
                         double de[2], double ds[2])
{
    if (mix == 2) {
        double s6 = pow(sa, 6.0) + pow(sb, 6.0);
        double e = 2.0 * sqrt(ea * eb) * sa * sa * sa * sb * sb * sb / s6;
        double sab = pow(0.5 * s6, 1.0 / 6.0);
        de[0] = e / (2.0 * ea);
        de[1] = e * (3.0 / sa - 6.0 * pow(sa, 5.0) / s6);
        ds[0] = 0.0;
        ds[1] = pow(sa, 5.0) / (2.0 * pow(sab, 5.0));
        return;
    }
    de[0] = 0.5 * sqrt(eb / ea);
    de[1] = 0.0;
    ds[0] = 0.0;
    ds[1] = mix == 1 ? 0.5 : 0.5 * sqrt(sb / sa);
}

/* Gradient of J = e_bar * E + sum_i g_i . F_i (E of Eq. 3, F_i = -dE/dx_i)
 * with respect to the per-type parameters (dtheta[P*ntypes + t], P = 0
 * eps_FG, 1 sigma_FG, 2 eps_CG, 3 sigma_CG) and the positions (dpos, n x 3).
 * Brute force over all non-excluded pairs i < j, serial.  Per pair, with
 * d = x_j - x_i, r = |d|, s = u~'(r)/r (F_i gets s d, F_j gets -s d):
 *   dJ/dx_j = e_bar u~' d/r + grad_d [ s (g_i - g_j) . d ],  dJ/dx_i = -dJ/dx_j,
 *   grad_d [ s w . d ] = s w + (ds/dr / r) (w . d) d,  ds/dr = u~''/r - u~'/r^2;
 *   dJ/dP = e_bar du~/dP + (du~'/dP / r) (g_i - g_j) . d,
 * and dJ/dP is carried to the per-type values through the mixing rule.  The
 * CG parameters of ordinary types receive nothing (Eq. 14 fixes their pair
 * parameters at zero).  Per-type parameters entering a geometric mean must be
 * positive.  Returns 0, or a negative code as oracle_setup.                 */
int oracle_grad(int n, const double *pos, const double *box, const int *types,
                const int *mol, int same_mol, const int *eoff, const int *eidx,
                int ntypes, const double *eps_fg, const double *sig_fg,
                const double *eps_cg, const double *sig_cg, int mix, const double cut[4],
                const double *cut_type, const double *cut_pair, int shift,
                const double *g, double e_bar, double *dtheta, double *dpos)
{
    size_t np = (size_t)ntypes * ntypes;
    double *table = (double *)malloc(sizeof(double) * np * OR_REC);
    double *dtab = (double *)malloc(sizeof(double) * np * 4 * OR_REC);
    double *w = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!table || !dtab || !w) { free(table); free(dtab); free(w); return -3; }
    int rc = oracle_setup(ntypes, eps_fg, sig_fg, eps_cg, sig_cg, mix, cut, cut_type, cut_pair,
                          shift, table);
    for (size_t k = 0; rc == 0 && k < np; ++k)
        for (int P = 0; P < 4 && rc == 0; ++P)
            rc = dparam_record(table + k * OR_REC, P, shift, dtab + (k * 4 + P) * OR_REC);
    if (rc) { free(table); free(dtab); free(w); return rc; }
    oracle_wrap(n, pos, box, w);
    memset(dtheta, 0, sizeof(double) * 4 * (size_t)ntypes);
    memset(dpos, 0, sizeof(double) * 3 * (size_t)n);
    const double *pe[4] = {eps_fg, sig_fg, eps_cg, sig_cg};
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            if (is_excluded(i, j, mol, same_mol, eoff, eidx)) continue;
            double d[3];
            min_image(w + 3 * i, w + 3 * j, box, d);      /* d = x_j - x_i */
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            int p = types[i], q = types[j];
            size_t k = (size_t)(p * ntypes + q);
            const double *R = table + k * OR_REC;
            if (!(r < R[R_CUT + 3])) continue;
            double u1;
            (void)oracle_pair(R, r, &u1, NULL);
            double u2 = pair_d2(R, r);
            double wv[3] = {g[3 * i] - g[3 * j], g[3 * i + 1] - g[3 * j + 1], g[3 * i + 2] - g[3 * j + 2]};
            double wd = wv[0] * d[0] + wv[1] * d[1] + wv[2] * d[2];
            double s = u1 / r;
            double dsr = (u2 / r - u1 / (r * r)) / r;
            for (int c = 0; c < 3; ++c) {
                double gj = e_bar * u1 * d[c] / r + s * wv[c] + dsr * wd * d[c];
                dpos[3 * j + c] += gj;
                dpos[3 * i + c] -= gj;
            }
            double cP[4];
            for (int P = 0; P < 4; ++P) {
                cP[P] = 0.0;
                if (P >= 2 && !(R[R_EPS_CG] > 0.0)) continue;
                double du, dup;
                pair_dparam(R, dtab + (k * 4 + P) * OR_REC, P, r, &du, &dup);
                cP[P] = e_bar * du + (dup / r) * wd;
            }
            /* through the mixing rule: (eps, sigma) of the FG pair (P = 0, 1)
             * and of the CG pair (P = 2, 3) to the per-type values            */
            for (int part = 0; part < 2; ++part) {
                if (part == 1 && !(R[R_EPS_CG] > 0.0)) continue;
                const double *E = pe[2 * part], *S = pe[2 * part + 1];
                double de[2], ds[2];
                mix_jacobian(mix, E[p], E[q], S[p], S[q], de, ds);
                for (int y = 0; y < 2; ++y)
                    dtheta[(2 * part + y) * ntypes + p] += cP[2 * part] * de[y] + cP[2 * part + 1] * ds[y];
                mix_jacobian(mix, E[q], E[p], S[q], S[p], de, ds);
                for (int y = 0; y < 2; ++y)
                    dtheta[(2 * part + y) * ntypes + q] += cP[2 * part] * de[y] + cP[2 * part + 1] * ds[y];
            }
        }
    free(table); free(dtab); free(w);
    return 0;
}

/*
 * md_oracle.c -- plain FP64 reference for the bonded terms of the paper's
 * molecular simulations (Sec. 3.2: AMBER_UA bonds, angles and Fourier
 * dihedrals next to the RelRes non-bonded terms).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the package smoke check and
 * the benchmark's CPU-baseline leg; nothing in the product library links or
 * calls it, and it shares no code with the HIP path.
 *
 * Readings (where Sec. 3.2 is silent):
 *   - The spring constants are those of the AMBER convention, without a
 *     factor 1/2: E_bond = K (r - r0)^2 and E_angle = K (theta - theta0)^2.
 *     The printed 180,640 zJ/nm^2 is exactly AMBER's 260 kcal/mol/A^2.
 *   - The Fourier dihedral is E = K (1 + cos(n phi - d)) with the IUPAC
 *     dihedral phi (trans = pi); for the paper's K (1 + cos 3 phi) the sign
 *     convention of phi does not matter.
 *   - Difference vectors inside a term use the single-shift minimum image
 *     (molecules are much smaller than half the box).
 *
 * Forces are -dE/dx written out from the geometry:
 *   bond:  d = x_i - x_j, r = |d|: F_i = -2K (r - r0) d / r, F_j = -F_i.
 *   angle: a = x_i - x_j, b = x_k - x_j, cos(theta) = a.b/(|a||b|):
 *          F_i = (dE/dtheta / sin theta) (b/|b| - cos(theta) a/|a|) / |a|,
 *          F_k likewise with a and b exchanged, F_j = -F_i - F_k.
 *   dihedral: b1 = x_j - x_i, b2 = x_k - x_j, b3 = x_l - x_k, m = b1 x b2,
 *          n = b2 x b3, phi = atan2(|b2| b1.n, m.n); with p = b1.b2/|b2|^2,
 *          q = b3.b2/|b2|^2 the gradients of phi are
 *          G_i = -|b2| m/|m|^2, G_l = |b2| n/|n|^2,
 *          G_j = -(1 + p) G_i + q G_l, G_k = p G_i - (1 + q) G_l,
 *          and F_x = -dE/dphi G_x.
 * The virial of a term is sum over its atoms of (x_atom - x_ref) (x) F_atom,
 * x_ref its second atom (the first for a bond), positions taken along the
 * term's minimum-image difference vectors.
 *
 * Build: with relres_oracle.c, gcc -O2 -std=c99 -fPIC -shared -fopenmp
 * -ffp-contract=off -lm
 */
#include <math.h>
#include <string.h>

static void mi_diff(const double *xa, const double *xb, const double *box, double d[3])
{
    /* d = x_a - x_b with the single-shift minimum image */
    for (int k = 0; k < 3; ++k) {
        double v = xa[k] - xb[k];
        double h = 0.5 * box[k];
        if (v > h) v -= box[k];
        else if (v < -h) v += box[k];
        d[k] = v;
    }
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static void add_virial(double *W, const double *lever, const double *f)
{
    W[0] += lever[0] * f[0];
    W[1] += lever[1] * f[1];
    W[2] += lever[2] * f[2];
    W[3] += lever[0] * f[1];
    W[4] += lever[0] * f[2];
    W[5] += lever[1] * f[2];
}

/* Energy of one dihedral and its angle (used by the tests as well). */
double oracle_dihedral_angle(const double *xi, const double *xj, const double *xk,
                             const double *xl, const double *box)
{
    double b1[3], b2[3], b3[3], m[3], n[3];
    mi_diff(xj, xi, box, b1);
    mi_diff(xk, xj, box, b2);
    mi_diff(xl, xk, box, b3);
    cross3(b1, b2, m);
    cross3(b2, b3, n);
    return atan2(sqrt(dot3(b2, b2)) * dot3(b1, n), dot3(m, n));
}

/* Bonded energy, forces and virial.  Forces are ADDED to F (n x 3);
 * E_out = {bonds, angles, dihedrals}; W_out {xx,yy,zz,xy,xz,yz} is added to.
 * bonds: nb x 2 atom indices with K, r0 per bond; angles: na x 3 (i, j, k;
 * j the vertex) with K, theta0; dihedrals: nd x 4 with K, n, d.           */
void oracle_bonded(int n_atoms, const double *pos, const double *box,
                   int nb, const int *bonds, const double *bk, const double *br0,
                   int na, const int *angles, const double *ak, const double *at0,
                   int nd, const int *dih, const double *dk, const int *dn, const double *dd,
                   double *F, double *E_out, double *W_out)
{
    (void)n_atoms;
    double eb = 0.0, ea = 0.0, ed = 0.0;
    for (int t = 0; t < nb; ++t) {
        int i = bonds[2 * t], j = bonds[2 * t + 1];
        double d[3];
        mi_diff(pos + 3 * i, pos + 3 * j, box, d);
        double r = sqrt(dot3(d, d));
        double dr = r - br0[t];
        eb += bk[t] * dr * dr;
        double s = -2.0 * bk[t] * dr / r;
        double fi[3] = {s * d[0], s * d[1], s * d[2]};
        for (int c = 0; c < 3; ++c) {
            F[3 * i + c] += fi[c];
            F[3 * j + c] -= fi[c];
        }
        add_virial(W_out, d, fi);
    }
    for (int t = 0; t < na; ++t) {
        int i = angles[3 * t], j = angles[3 * t + 1], k = angles[3 * t + 2];
        double a[3], b[3];
        mi_diff(pos + 3 * i, pos + 3 * j, box, a);
        mi_diff(pos + 3 * k, pos + 3 * j, box, b);
        double la = sqrt(dot3(a, a)), lb = sqrt(dot3(b, b));
        double c = dot3(a, b) / (la * lb);
        if (c > 1.0) c = 1.0;
        if (c < -1.0) c = -1.0;
        double th = acos(c);
        double dth = th - at0[t];
        ea += ak[t] * dth * dth;
        double dE = 2.0 * ak[t] * dth;
        double sn = sin(th);
        double g = dE / sn;
        double fi[3], fk[3];
        for (int q = 0; q < 3; ++q) {
            fi[q] = g * (b[q] / lb - c * a[q] / la) / la;
            fk[q] = g * (a[q] / la - c * b[q] / lb) / lb;
        }
        for (int q = 0; q < 3; ++q) {
            F[3 * i + q] += fi[q];
            F[3 * k + q] += fk[q];
            F[3 * j + q] -= fi[q] + fk[q];
        }
        add_virial(W_out, a, fi);
        add_virial(W_out, b, fk);
    }
    for (int t = 0; t < nd; ++t) {
        int i = dih[4 * t], j = dih[4 * t + 1], k = dih[4 * t + 2], l = dih[4 * t + 3];
        double b1[3], b2[3], b3[3], m[3], nn[3];
        mi_diff(pos + 3 * j, pos + 3 * i, box, b1);
        mi_diff(pos + 3 * k, pos + 3 * j, box, b2);
        mi_diff(pos + 3 * l, pos + 3 * k, box, b3);
        cross3(b1, b2, m);
        cross3(b2, b3, nn);
        double lb2 = sqrt(dot3(b2, b2));
        double phi = atan2(lb2 * dot3(b1, nn), dot3(m, nn));
        double arg = dn[t] * phi - dd[t];
        ed += dk[t] * (1.0 + cos(arg));
        double dE = -dk[t] * dn[t] * sin(arg);
        double mm = dot3(m, m), n2 = dot3(nn, nn);
        double p = dot3(b1, b2) / (lb2 * lb2), q = dot3(b3, b2) / (lb2 * lb2);
        double Gi[3], Gl[3], Gj[3], Gk[3];
        for (int c = 0; c < 3; ++c) {
            Gi[c] = -lb2 * m[c] / mm;
            Gl[c] = lb2 * nn[c] / n2;
        }
        for (int c = 0; c < 3; ++c) {
            Gj[c] = -(1.0 + p) * Gi[c] + q * Gl[c];
            Gk[c] = p * Gi[c] - (1.0 + q) * Gl[c];
        }
        double fi[3], fj[3], fk[3], fl[3];
        for (int c = 0; c < 3; ++c) {
            fi[c] = -dE * Gi[c];
            fj[c] = -dE * Gj[c];
            fk[c] = -dE * Gk[c];
            fl[c] = -dE * Gl[c];
            F[3 * i + c] += fi[c];
            F[3 * j + c] += fj[c];
            F[3 * k + c] += fk[c];
            F[3 * l + c] += fl[c];
        }
        /* levers from x_j: x_i - x_j = -b1, x_k - x_j = b2, x_l - x_j = b2 + b3 */
        double li[3] = {-b1[0], -b1[1], -b1[2]};
        double ll[3] = {b2[0] + b3[0], b2[1] + b3[1], b2[2] + b3[2]};
        add_virial(W_out, li, fi);
        add_virial(W_out, b2, fk);
        add_virial(W_out, ll, fl);
    }
    E_out[0] = eb;
    E_out[1] = ea;
    E_out[2] = ed;
}

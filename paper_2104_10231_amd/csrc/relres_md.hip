// relres_md.hip -- gfx950 kernels of the molecular model around the RelRes
// pair potential (Sec. 3.2 of the paper): bonded terms, scaled 1-4 pairs and
// a Nose-Hoover velocity-Verlet integrator.
//
// Bonded terms: a group of lanes per atom evaluates the atom's (term, slot)
// entries and scaled 1-4 pairs side by side in FP64 and sums their forces
// with lane moves in a fixed order; in a dynamics step the same kernel gives
// the half kick.  A term's energy and virial are counted by its first slot.
// No atomics, so results are deterministic.  Formulas
// (forces are -dE/dx):
//   bond      E = K (r - r0)^2, d = x_i - x_j: F_i = -2K (r - r0) d / r
//   angle     E = K (theta - theta0)^2, a = x_i - x_j, b = x_k - x_j:
//             F_i = (dE/dtheta / sin theta)(b/|b| - cos(theta) a/|a|)/|a|,
//             F_k likewise with a and b exchanged, F_j = -F_i - F_k
//   dihedral  E = K (1 + cos(n phi - d)), b1 = x_j - x_i, b2 = x_k - x_j,
//             b3 = x_l - x_k, m = b1 x b2, n = b2 x b3,
//             phi = atan2(|b2| b1.n, m.n); p = b1.b2/|b2|^2, q = b3.b2/|b2|^2;
//             dphi/dx_i = -|b2| m/|m|^2, dphi/dx_l = |b2| n/|n|^2,
//             dphi/dx_j = -(1 + p) dphi/dx_i + q dphi/dx_l,
//             dphi/dx_k = p dphi/dx_i - (1 + q) dphi/dx_l
// (the gradient of phi as in Blondel and Karplus, J. Comput. Chem. 17, 1132
// (1996)).  1-4 pairs: the pair potential of Eq. 20 of the pair (FG and CG
// parts, the pair's own distances) times the 1-4 factor.
#include "relres_internal.h"
#include "relres_pair.h"
#include "relres_lanes.h"

namespace relres {
namespace {

constexpr int kMdBlock = 256;

// d = x_a - x_b with the single-shift minimum image, from positions already
// read.  The shift is taken by selects (both shifted values computed), so the
// same roundings as subtracting or adding the box under a branch.
__device__ __forceinline__ void mi_diff(const double xa[3], const double xb[3],
                                        const double box[3], double d[3])
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double v = xa[k] - xb[k];
        const double h = 0.5 * box[k];
        const double lo = v - box[k], hi = v + box[k];
        d[k] = v > h ? lo : (v < -h ? hi : v);
    }
}

// The positions of an item's atoms i, j, k, l (unused ones, and the padding
// items' atoms, read as atom 0 and ignored), all read before any is used.
__device__ __forceinline__ void item_positions(const double* __restrict__ pos, int n,
                                               const BondItem& it, double x[4][3])
{
    const int at[4] = {it.i, it.j, it.k, it.l};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int a = (unsigned)at[q] < (unsigned)n ? at[q] : 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) x[q][c] = pos[3 * (size_t)a + c];
    }
}

__device__ __forceinline__ double dot3(const double* a, const double* b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

__device__ __forceinline__ void cross3(const double* a, const double* b, double* c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ void add_virial(double* w, const double* lever, const double* f)
{
    w[0] += lever[0] * f[0];
    w[1] += lever[1] * f[1];
    w[2] += lever[2] * f[2];
    w[3] += lever[0] * f[1];
    w[4] += lever[0] * f[2];
    w[5] += lever[1] * f[2];
}

// Fixed-order sum over the block (kMdBlock threads) of v[0..K): the result
// lands in threads 0..K-1 (component threadIdx.x).  Lane moves within each
// wave (the K chains interleaved), then the waves' sums through LDS: two
// block barriers, where a tree through LDS takes one per halving.
template <int K>
__device__ __forceinline__ double block_sum(const double* v, double (*red)[kMdBlock / 64])
{
    double s[K];
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = v[k];
    wave_sums(s);                      // complete in lane 63
    const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
    if (lane == 63) {
#pragma unroll
        for (int k = 0; k < K; ++k) red[k][w] = s[k];
    }
    __syncthreads();
    double r = 0.0;
    if ((int)threadIdx.x < K)
        for (int q = 0; q < kMdBlock / 64; ++q) r += red[threadIdx.x][q];
    __syncthreads();
    return r;
}

// The force of one (term, slot) entry on its atom, added to fa; the term's
// energy and virial go to acc (energies 0..2, virial 4..9) from its first
// slot only.
__device__ __forceinline__ void entry_force(const BondedArgs& b, const BondItem& it,
                                            const double x[4][3], double fa[3], double acc[10])
{
    const int kind = it.kind, slot = it.slot, t = it.par;
    double f[4][3];
    if (kind == 0) {
        const double2 par = b.bond_par[t];
        double d[3];
        mi_diff(x[0], x[1], b.box, d);
        const double r = sqrt(dot3(d, d));
        const double dr = r - par.y;
        const double sc = -2.0 * par.x * dr / r;
        for (int c = 0; c < 3; ++c) {
            f[0][c] = sc * d[c];
            f[1][c] = -f[0][c];
        }
        if (slot == 0) {
            acc[0] += par.x * dr * dr;
            add_virial(acc + 4, d, f[0]);
        }
    } else if (kind == 1) {
        const double2 par = b.angle_par[t];
        double u[3], v[3];
        mi_diff(x[0], x[1], b.box, u);
        mi_diff(x[2], x[1], b.box, v);
        // reciprocals once: a divide is a long instruction sequence in FP64
        const double ilu = 1.0 / sqrt(dot3(u, u)), ilv = 1.0 / sqrt(dot3(v, v));
        double c = dot3(u, v) * ilu * ilv;
        c = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
        const double th = acos(c);
        const double dth = th - par.y;
        const double g = 2.0 * par.x * dth / sqrt((1.0 - c) * (1.0 + c));   // sin theta
        for (int q = 0; q < 3; ++q) {
            f[0][q] = g * (v[q] * ilv - c * u[q] * ilu) * ilu;
            f[2][q] = g * (u[q] * ilu - c * v[q] * ilv) * ilv;
            f[1][q] = -f[0][q] - f[2][q];
        }
        if (slot == 0) {
            acc[1] += par.x * dth * dth;
            add_virial(acc + 4, u, f[0]);
            add_virial(acc + 4, v, f[2]);
        }
    } else {
        const double4 par = b.dih_par[t];      // K, n, cos d, sin d
        double b1[3], b2[3], b3[3], m[3], nn[3];
        mi_diff(x[1], x[0], b.box, b1);
        mi_diff(x[2], x[1], b.box, b2);
        mi_diff(x[3], x[2], b.box, b3);
        cross3(b1, b2, m);
        cross3(b2, b3, nn);
        const double lb2 = sqrt(dot3(b2, b2));
        // phi = atan2(y, x) without the library calls: cos phi = x / r,
        // sin phi = y / r (r = |m||n|), cos and sin of n phi by repeated
        // angle addition, then of n phi - d with cos d, sin d from the host
        const double x = dot3(m, nn), y = lb2 * dot3(b1, nn);
        const double ir = 1.0 / sqrt(x * x + y * y);
        const double cp = x * ir, sp = y * ir;
        double cn = 1.0, sn = 0.0;
        for (int k = 0; k < (int)par.y; ++k) {
            const double c2 = cn * cp - sn * sp;
            sn = sn * cp + cn * sp;
            cn = c2;
        }
        const double cos_arg = cn * par.z + sn * par.w;
        const double sin_arg = sn * par.z - cn * par.w;
        const double dE = -par.x * par.y * sin_arg;
        const double imm = lb2 / dot3(m, m), in2 = lb2 / dot3(nn, nn);
        const double ib2 = 1.0 / (lb2 * lb2);
        const double p = dot3(b1, b2) * ib2, q = dot3(b3, b2) * ib2;
        for (int c = 0; c < 3; ++c) {
            const double gi = -m[c] * imm, gl = nn[c] * in2;
            f[0][c] = -dE * gi;
            f[3][c] = -dE * gl;
            f[1][c] = -dE * (-(1.0 + p) * gi + q * gl);
            f[2][c] = -dE * (p * gi - (1.0 + q) * gl);
        }
        if (slot == 0) {
            acc[2] += par.x * (1.0 + cos_arg);
            const double li[3] = {-b1[0], -b1[1], -b1[2]};
            const double ll[3] = {b2[0] + b3[0], b2[1] + b3[1], b2[2] + b3[2]};
            add_virial(acc + 4, li, f[0]);
            add_virial(acc + 4, b2, f[2]);
            add_virial(acc + 4, ll, f[3]);
        }
    }
    for (int c = 0; c < 3; ++c) fa[c] += f[slot][c];
}

// The scaled 1-4 pair (a, j) through Eq. 20 (FG and CG parts, the pair's own
// distances), seen from atom a: its force on a added to fa, half its energy
// to acc[3] and half its virial to acc[4..9] (the pair is met from both atoms).
__device__ __forceinline__ void pair14_force(const BondedArgs& b, const BondItem& it,
                                             const double x[4][3], double fa[3], double acc[10])
{
    double d[3];
    mi_diff(x[0], x[1], b.box, d);             // x_a - x_j
    const double r2 = dot3(d, d);
    const int pi = it.par;
    const Cutoffs<double>& cut = b.pcut64[pi];
    double fp = 0.0, en = 0.0;
    if (r2 < cut.rso2) {
        double f1, e1;
        fg_term<MathF64<2>>(b.coef64[pi], cut, r2, f1, e1);
        fp += f1;
        en += e1;
    }
    if (r2 < cut.rco2) {
        double f2, e2;
        cg_term<MathF64<2>>(b.coef64[pi], cut, r2, f2, e2);
        fp += f2;
        en += e2;
    }
    const double s = b.scale14 * fp;           // F_a = s (x_a - x_j)
    const double f[3] = {s * d[0], s * d[1], s * d[2]};
    for (int c = 0; c < 3; ++c) fa[c] += f[c];
    acc[3] += 0.5 * b.scale14 * en;
    const double hd[3] = {0.5 * d[0], 0.5 * d[1], 0.5 * d[2]};
    add_virial(acc + 4, hd, f);
}

// Bonded and 1-4 forces, one aligned group of 2^log_lanes lanes per atom:
// the lanes take the atom's items (its term entries in order, then its 1-4
// partners; one padded record each, so a lane needs no offset table) in
// turn, and the group adds their forces with lane moves in a fixed order, so
// an atom's items are evaluated side by side and no force passes through
// memory.  The group's first lane adds the sum to `forces`
// and, in a dynamics step (kick != 0), gives the half kick v += dt/2 F/m and
// the kinetic term of the block partial.  With b.partial every block writes
// its 10 sums (energies: bonds, angles, dihedrals, 1-4; virial).  No
// atomics, so results are deterministic.
template <typename TF>
__global__ __launch_bounds__(kMdBlock) void k_bonded(BondedArgs b, MdArgs m, int kick)
{
    __shared__ double red[10][kMdBlock / 64];
    const int lg = b.log_lanes;
    const int G = 1 << lg;
    const int gid = blockIdx.x * kMdBlock + (int)threadIdx.x;
    const int a = gid >> lg;
    const int sub = gid & (G - 1);
    double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    double fa[3] = {0.0, 0.0, 0.0};
    const bool live = a < b.n;
    const bool lead = live && sub == 0;
    // the leader's own data first: it does not depend on the items
    TF* F = (TF*)b.forces;
    TF f0[3] = {TF(0), TF(0), TF(0)};
    double v0[3] = {0.0, 0.0, 0.0}, ma = 1.0;
    if (lead) {
        for (int c = 0; c < 3; ++c) f0[c] = F[3 * a + c];
        if (kick) {
            for (int c = 0; c < 3; ++c) v0[c] = m.vel[3 * a + c];
            ma = m.mass[a];
        }
    }
    if (live) {
        const BondItem* items = b.items + (size_t)a * b.slots;
        for (int k = sub; k < b.slots; k += G) {
            const BondItem it = items[k];
            double x[4][3];
            item_positions(b.pos, b.n, it, x);
            if (it.kind == 3) pair14_force(b, it, x, fa, acc);
            else if (it.kind >= 0) entry_force(b, it, x, fa, acc);
        }
    }
    // every lane takes part in the group sums (idle lanes add zeros)
    for (int c = 0; c < 3; ++c) fa[c] = group_sum(fa[c], G);
    double ke = 0.0;
    if (lead) {
        TF ft[3];
        for (int c = 0; c < 3; ++c) {
            ft[c] = f0[c] + (TF)fa[c];
            F[3 * a + c] = ft[c];
        }
        if (kick) {
            const double dt = m.st->dt;
            const double am = m.ftm2v / ma;
            for (int c = 0; c < 3; ++c) {
                const double v = v0[c] + 0.5 * dt * am * (double)ft[c];
                m.vel[3 * a + c] = v;
                ke += ma * v * v;
            }
        }
    }
    if (b.partial) {
        const double r = block_sum<10>(acc, red);
        if (threadIdx.x < 10) b.partial[(size_t)blockIdx.x * 10 + threadIdx.x] = r;
    }
    if (kick) {
        const double r = block_sum<1>(&ke, red);
        if (threadIdx.x == 0) m.partial[blockIdx.x] = r;
    }
}

// Sum over the blocks' partials in a fixed order: lane l of a wave adds
// blocks l, l + 64, ... of p1 and then of p2, and the wave adds its lanes.
// A lane's loads are issued kSumLoads at a time before any is added, so a
// few hundred partials cost one or two memory round trips, not one per
// block of the lane.
constexpr int kSumLoads = 8;

__device__ __forceinline__ void add_blocks(const double* __restrict__ p, int n, int K, int k,
                                           int lane, double& s)
{
    auto round = [&](int base) {
        double x[kSumLoads];
#pragma unroll
        for (int u = 0; u < kSumLoads; ++u) {
            const int blk = base + 64 * u;
            x[u] = blk < n ? p[(size_t)blk * K + k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kSumLoads; ++u)
            if (base + 64 * u < n) s += x[u];
    };
    // the first round outside the loop: its reads are not held back until
    // the caller's earlier reads are in
    if (lane < n) round(lane);
    for (int base = lane + 64 * kSumLoads; base < n; base += 64 * kSumLoads) round(base);
}

__device__ __forceinline__ double sum_blocks(const double* __restrict__ p1, int n1,
                                             const double* __restrict__ p2, int n2, int K, int k)
{
    const int lane = (int)threadIdx.x & 63;
    double s = 0.0;
    add_blocks(p1, n1, K, k, lane, s);
    add_blocks(p2, n2, K, k, lane, s);
    return wave_sum(s);                // complete in lane 63
}

// out[k] = the sums over blocks of p1[blk * K + k] and of p2 (one wave per
// component k).
__global__ void k_sum_partials(const double* __restrict__ p1, int n1,
                               const double* __restrict__ p2, int n2, int K,
                               double* __restrict__ out)
{
    const int k = (int)threadIdx.x >> 6;
    const double s = sum_blocks(p1, n1, p2, n2, K, k);
    if (((int)threadIdx.x & 63) == 63) out[k] = s;
}

// ---------------------------------------------------------------------------
// Nose-Hoover velocity Verlet.  Stored velocities v_s; the true velocities
// are v_s * st.s2 (the scale of the last thermostat half step, applied
// together with the next one).  Thermostat half step over dt/2:
//   xi += dt/4 G(K);  v *= exp(-xi dt/2) (K *= its square);  eta += dt/2 xi;
//   xi += dt/4 G(K),   G(K) = (2K - g kT)/Q.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void thermostat_half(MdState* st)
{
    const double dt = st->dt;
    st->xi += 0.25 * dt * (2.0 * st->K - st->g * st->kT) / st->Q;
    const double s = exp(-st->xi * 0.5 * dt);
    st->K *= s * s;
    st->eta += 0.5 * dt * st->xi;
    st->xi += 0.25 * dt * (2.0 * st->K - st->g * st->kT) / st->Q;
    st->s_last = s;
}

// The scalar work between two steps on a copy of the state: the kinetic
// energy from the partial sum; with `second` the second thermostat half
// step of the step just done (and, with `row`, its thermodynamic output: the
// non-bonded energy of Eq. 3, the 1-4, bond, angle and dihedral energies,
// the kinetic energy, the extended energy K + U + Q xi^2/2 + g kT eta and
// the trace of the virial); with `first` the first half step of the next
// step, whose drift applies s2 s1 to the stored velocities.
__device__ void scalar_step(MdState& st, double ksum, double ftm2v, int second, int first,
                            const double* __restrict__ e_nb, const double* __restrict__ w_nb,
                            const double* __restrict__ eb, double* __restrict__ row)
{
    st.K = 0.5 * ksum / ftm2v;
    if (second) {
        thermostat_half(&st);
        st.s2 = st.s_last;
        if (row) {
            const double u = e_nb[0] + eb[3] + eb[0] + eb[1] + eb[2];
            row[0] = e_nb[0];
            row[1] = eb[3];
            row[2] = eb[0];
            row[3] = eb[1];
            row[4] = eb[2];
            row[5] = st.K;
            row[6] = st.K + u + 0.5 * st.Q * st.xi * st.xi + st.g * st.kT * st.eta;
            row[7] = w_nb[0] + w_nb[1] + w_nb[2] + eb[4] + eb[5] + eb[6];
        }
    }
    if (first) {
        thermostat_half(&st);
        st.s_apply = st.s2 * st.s_last;
        st.s2 = 1.0;
    }
}

// Drift of one step.  With `scalar`, every block first does the scalar work
// between the previous step and this one (the same sums in the same order,
// so every block gets the same state; block 0 stores it in st_out and writes
// the row), which saves a launch per step; st_in is not written, so no block
// can see a half-updated state.  Without it the state in st_in is current.
template <typename TF>
__global__ __launch_bounds__(kMdBlock) void k_md_drift(MdArgs m, const MdState* st_in,
                                                       MdState* st_out, int nparts, int scalar,
                                                       const double* __restrict__ e_nb,
                                                       const double* __restrict__ w_nb,
                                                       const double* __restrict__ eb,
                                                       double* __restrict__ row)
{
    __shared__ double s_sh;
    // the atom's data first: none of it depends on the scalar work, so its
    // reads overlap the sum of the partials
    const int i = blockIdx.x * kMdBlock + threadIdx.x;
    const bool in = i < m.n;
    const TF* F = (const TF*)m.forces;
    double v0[3] = {0.0, 0.0, 0.0}, x0[3] = {0.0, 0.0, 0.0}, xr[3] = {0.0, 0.0, 0.0};
    TF f0[3] = {TF(0), TF(0), TF(0)};
    double mass = 1.0;
    if (in) {
        for (int c = 0; c < 3; ++c) {
            v0[c] = m.vel[3 * i + c];
            x0[c] = m.pos[3 * i + c];
            xr[c] = m.xref[3 * i + c];
            f0[c] = F[3 * i + c];
        }
        mass = m.mass[i];
    }
    const double dt = st_in->dt;
    double s;
    if (scalar) {
        if (threadIdx.x < 64) {
            const double ks = sum_blocks(m.partial, nparts, nullptr, 0, 1, 0);
            if (threadIdx.x == 63) {
                MdState st = *st_in;
                scalar_step(st, ks, m.ftm2v, 1, 1, e_nb, w_nb, eb,
                            blockIdx.x == 0 ? row : nullptr);
                if (blockIdx.x == 0) *st_out = st;
                s_sh = st.s_apply;
            }
        }
        __syncthreads();
        s = s_sh;
    } else {
        s = st_in->s_apply;
    }
    if (!in) return;
    const double am = m.ftm2v / mass;
    double dmax2 = 0.0;
    for (int c = 0; c < 3; ++c) {
        const double v = v0[c] * s + 0.5 * dt * am * (double)f0[c];
        m.vel[3 * i + c] = v;
        const double x = x0[c] + dt * v;
        m.pos[3 * i + c] = x;
        const double dx = x - xr[c];
        dmax2 += dx * dx;
    }
    // an atom that moved more than half the skin since the last build
    // invalidates the lists; the host checks the flag at the next build
    if (dmax2 > m.half_skin2) atomicOr(m.stale, 1u);
}

// Kinetic partials of the stored velocities (no kick), at the start of a run.
__global__ __launch_bounds__(kMdBlock) void k_md_kinetic(MdArgs m)
{
    __shared__ double red[1][kMdBlock / 64];
    const int i = blockIdx.x * kMdBlock + threadIdx.x;
    double ke = 0.0;
    if (i < m.n)
        for (int c = 0; c < 3; ++c) ke += m.mass[i] * m.vel[3 * i + c] * m.vel[3 * i + c];
    const double r = block_sum<1>(&ke, red);
    if (threadIdx.x == 0) m.partial[blockIdx.x] = r;
}

// The scalar work between two steps as a kernel of its own (one wave; at
// the start and the end of a run, where no drift follows): scalar_step on
// the state in place.
__global__ void k_md_scalar(MdState* st, const double* __restrict__ partial, int nblocks,
                            double ftm2v, int second, int first, const double* __restrict__ e_nb,
                            const double* __restrict__ w_nb, const double* __restrict__ eb,
                            double* __restrict__ row)
{
    // one wave: the block partials in a fixed order, then lane 63 alone
    const double s = sum_blocks(partial, nblocks, nullptr, 0, 1, 0);
    if (threadIdx.x != 63) return;
    MdState cur = *st;
    scalar_step(cur, s, ftm2v, second, first, e_nb, w_nb, eb, row);
    *st = cur;
}

// Make the stored velocities the true ones (v_s *= s2), at the end of a run.
__global__ __launch_bounds__(kMdBlock) void k_md_finish(MdArgs m)
{
    const int i = blockIdx.x * kMdBlock + threadIdx.x;
    if (i >= m.n) return;
    const double s = m.st->s2;
    for (int c = 0; c < 3; ++c) m.vel[3 * i + c] *= s;
}

__global__ void k_md_unit_scale(MdState* st) { st->s2 = 1.0; }

}  // namespace

hipError_t launch_bonded(const BondedArgs& b, const MdArgs* m, int force_prec, hipStream_t s)
{
    if (b.n == 0) return hipSuccess;
    const dim3 grid(bonded_blocks(b.n, b.log_lanes));
    const MdArgs none{};
    const int kick = m ? 1 : 0;
    if (force_prec == 64)
        hipLaunchKernelGGL(k_bonded<double>, grid, dim3(kMdBlock), 0, s, b, m ? *m : none, kick);
    else
        hipLaunchKernelGGL(k_bonded<float>, grid, dim3(kMdBlock), 0, s, b, m ? *m : none, kick);
    return hipGetLastError();
}

int md_blocks(int n) { return (n + kMdBlock - 1) / kMdBlock; }

int bonded_blocks(int n, int log_lanes)
{
    return (int)(((long long)n << log_lanes) + kMdBlock - 1) / kMdBlock;
}

hipError_t launch_sum_partials(const double* p1, int n1, const double* p2, int n2, int K,
                               double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64 * K), 0, s, p1, n1, p2, n2, K, out);
    return hipGetLastError();
}

hipError_t launch_md_drift(const MdArgs& m, const MdState* st_in, MdState* st_out, int nparts,
                           int scalar, const double* e_nb, const double* w_nb, const double* eb,
                           double* row, int force_prec, hipStream_t s)
{
    const int blocks = (m.n + kMdBlock - 1) / kMdBlock;
    if (force_prec == 64)
        hipLaunchKernelGGL(k_md_drift<double>, dim3(blocks), dim3(kMdBlock), 0, s, m, st_in,
                           st_out, nparts, scalar, e_nb, w_nb, eb, row);
    else
        hipLaunchKernelGGL(k_md_drift<float>, dim3(blocks), dim3(kMdBlock), 0, s, m, st_in,
                           st_out, nparts, scalar, e_nb, w_nb, eb, row);
    return hipGetLastError();
}

hipError_t launch_md_kinetic(const MdArgs& m, hipStream_t s)
{
    hipLaunchKernelGGL(k_md_kinetic, dim3((m.n + kMdBlock - 1) / kMdBlock), dim3(kMdBlock), 0, s, m);
    return hipGetLastError();
}

hipError_t launch_md_scalar(MdState* st, const double* partial, int nblocks, double ftm2v,
                            int second, int first, const double* e_nb, const double* w_nb,
                            const double* eb, double* row, hipStream_t s)
{
    hipLaunchKernelGGL(k_md_scalar, dim3(1), dim3(64), 0, s, st, partial, nblocks, ftm2v, second,
                       first, e_nb, w_nb, eb, row);
    return hipGetLastError();
}

hipError_t launch_md_finish(const MdArgs& m, hipStream_t s)
{
    const int blocks = (m.n + kMdBlock - 1) / kMdBlock;
    hipLaunchKernelGGL(k_md_finish, dim3(blocks), dim3(kMdBlock), 0, s, m);
    hipLaunchKernelGGL(k_md_unit_scale, dim3(1), dim3(1), 0, s, m.st);
    return hipGetLastError();
}

}  // namespace relres

// relres_kernels.hip -- gfx950 kernels of the RelRes Lennard-Jones hot path.
//
// Build (every rebuild):  k_bin -> k_scan -> k_scatter -> k_cellsort -> k_lists
//   Two cell grids are built side by side: the atom grid (cells >= r_s+ + skin,
//   all atoms) and the site grid (cells >= r_c+ + skin, hybrid atoms only).
//   Cells are numbered in Morton order so that neighbouring cells, and the
//   atoms they hold, sit close together in memory.  Within a cell, members are
//   ordered by caller index, which makes every list row deterministic.
//   k_lists stages the candidate atoms of the deduplicated 27-cell stencil in
//   LDS, one wave tests 64 candidates of one home atom at a time and appends
//   the survivors to that atom's row with a ballot + mbcnt prefix.
// Forces (every call): k_forces
//   One launch covers both lists.  Rows of ordinary atoms take the FG part over
//   their atom-list row; rows of hybrid atoms take the FG part over their
//   atom-list row plus the CG part over their site-list row.  Each row is owned
//   by a group of lanes that accumulate its force in registers and reduce it
//   with cross-lane shuffles, so no force atomics are needed.  Energy and
//   virial are accumulated in FP64 and reduced in a fixed order by the last
//   block to finish.
#include "relres_internal.h"

namespace relres {
namespace {

constexpr int kWave = 64;
constexpr int kChunk = 256;    // candidates staged in LDS per pass
constexpr int kHomeMax = 256;  // home atoms whose counters live in LDS at once

// Wrap one coordinate into [0, L):  w = x - L floor(x / L), fixed into range.
// Separately rounded operations; the oracle performs the same sequence.
__device__ __forceinline__ double wrap_coord(double x, double L)
{
#pragma clang fp contract(off)
    double w = x - L * floor(x / L);
    if (w < 0.0) w += L;
    if (w >= L) w -= L;
    if (w < 0.0 || w >= L) w = 0.0;
    return w;
}

__device__ __forceinline__ int cell_coord(double w, double inv, int n)
{
    int c = (int)(w * inv);
    return c < n ? c : n - 1;
}

// List membership in FP64 on wrapped positions (a = home atom, b = candidate):
// single-shift minimum image, r2 = (dx dx + dy dy) + dz dz, strict r2 < rl2.
__device__ __forceinline__ bool member(const double4 a, const double4 b, double Lx, double Ly,
                                       double Lz, double hx, double hy, double hz, double rl2)
{
#pragma clang fp contract(off)
    double dx = b.x - a.x;
    if (dx > hx) dx -= Lx; else if (dx < -hx) dx += Lx;
    double dy = b.y - a.y;
    if (dy > hy) dy -= Ly; else if (dy < -hy) dy += Ly;
    double dz = b.z - a.z;
    if (dz > hz) dz -= Lz; else if (dz < -hz) dz += Lz;
    double r2 = (dx * dx + dy * dy) + dz * dz;
    return r2 < rl2;
}

__device__ __forceinline__ int lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ---------------------------------------------------------------------------
// build kernels
// ---------------------------------------------------------------------------

__global__ void k_bin(int n, const double* __restrict__ pos, double Lx, double Ly, double Lz,
                      TopoDev topo, const GridDev* __restrict__ grids,
                      double4* __restrict__ wpos, int2* __restrict__ key_a,
                      int2* __restrict__ key_s, Status* __restrict__ st)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
        atomicOr(&st->nonfinite, 1);
        x = y = z = 0.0;
    }
    const double wx = wrap_coord(x, Lx), wy = wrap_coord(y, Ly), wz = wrap_coord(z, Lz);
    wpos[i] = make_double4(wx, wy, wz, 0.0);
    {
        const GridDev& g = grids[0];
        const int lin = (cell_coord(wx, g.inv_cell[0], g.n[0]) * g.n[1] +
                         cell_coord(wy, g.inv_cell[1], g.n[1])) * g.n[2] +
                        cell_coord(wz, g.inv_cell[2], g.n[2]);
        const int r = g.rank_of_lin[lin];
        key_a[i] = make_int2(r, atomicAdd(&g.count[r], 1));
    }
    if (topo.hybrid[topo.types[i]]) {
        const GridDev& g = grids[1];
        const int lin = (cell_coord(wx, g.inv_cell[0], g.n[0]) * g.n[1] +
                         cell_coord(wy, g.inv_cell[1], g.n[1])) * g.n[2] +
                        cell_coord(wz, g.inv_cell[2], g.n[2]);
        const int r = g.rank_of_lin[lin];
        key_s[i] = make_int2(r, atomicAdd(&g.count[r], 1));
    } else {
        key_s[i] = make_int2(-1, -1);
    }
}

// One block per grid: exclusive scan of the per-cell counts into `start`,
// then the counts are cleared for the next build.  Counts are staged through
// LDS in segments of kScanSeg cells with coalesced loads; each thread scans a
// contiguous run of its segment.  Block 0 also clears the list statistics.
constexpr int kScanThreads = 1024;
constexpr int kScanSeg = 8192;
__global__ __launch_bounds__(kScanThreads) void k_scan(GridDev* __restrict__ grids,
                                                       Status* __restrict__ st)
{
    __shared__ int vals[kScanSeg];
    __shared__ int sums[kScanThreads];
    __shared__ int carry_sh;
    if (blockIdx.x == 0 && threadIdx.x < 2 * kStatSlots) {
        const int g = threadIdx.x / kStatSlots, k = threadIdx.x % kStatSlots;
        st->max_row[g][k] = 0;
        st->entries[g][k] = 0ull;
    }
    const GridDev& g = grids[blockIdx.x];
    const int nc = g.ncell;
    const int t = threadIdx.x;
    constexpr int per = kScanSeg / kScanThreads;
    if (t == 0) carry_sh = 0;
    for (int seg = 0; seg < nc; seg += kScanSeg) {
        const int len = min(kScanSeg, nc - seg);
        for (int k = t; k < kScanSeg; k += kScanThreads) vals[k] = k < len ? g.count[seg + k] : 0;
        __syncthreads();
        int s = 0;
#pragma unroll
        for (int k = 0; k < per; ++k) s += vals[t * per + k];
        sums[t] = s;
        __syncthreads();
        for (int off = 1; off < kScanThreads; off <<= 1) {
            const int v = t >= off ? sums[t - off] : 0;
            __syncthreads();
            sums[t] += v;
            __syncthreads();
        }
        int run = carry_sh + sums[t] - s;
#pragma unroll
        for (int k = 0; k < per; ++k) {
            const int v = vals[t * per + k];
            vals[t * per + k] = run;
            run += v;
        }
        __syncthreads();
        for (int k = t; k < len; k += kScanThreads) {
            g.start[seg + k] = vals[k];
            g.count[seg + k] = 0;
        }
        if (t == kScanThreads - 1) carry_sh += sums[kScanThreads - 1];
        __syncthreads();
    }
    if (t == 0) g.start[nc] = carry_sh;
}

__global__ void k_scatter(int n, const GridDev* __restrict__ grids, const int2* __restrict__ key_a,
                          const int2* __restrict__ key_s)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int2 ka = key_a[i];
    grids[0].user_unsorted[grids[0].start[ka.x] + ka.y] = i;
    const int2 ks = key_s[i];
    if (ks.x >= 0) grids[1].user_unsorted[grids[1].start[ks.x] + ks.y] = i;
}

// One wave per cell: order the members of the cell by caller index (rank by
// counting) and write the sorted position / (type, molecule) / index arrays.
__global__ void k_cellsort(const GridDev* __restrict__ grids, int ncell_a, int ncell_total,
                           const double4* __restrict__ wpos, TopoDev topo,
                           int* __restrict__ user2arow)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int nwaves = (gridDim.x * blockDim.x) / kWave;
    for (int cell = wave; cell < ncell_total; cell += nwaves) {
        const bool site = cell >= ncell_a;
        const GridDev& g = grids[site ? 1 : 0];
        const int c = site ? cell - ncell_a : cell;
        const int b = g.start[c];
        const int len = g.start[c + 1] - b;
        if (len <= kWave) {
            // rank by counting with cross-lane reads, no memory traffic
            const int u = lane < len ? g.user_unsorted[b + lane] : 0x7fffffff;
            int r = 0;
            for (int k = 0; k < len; ++k) r += __shfl(u, k) < u;
            if (lane < len) {
                const int dst = b + r;
                g.user[dst] = u;
                g.pos[dst] = wpos[u];
                g.meta[dst] = make_int2(topo.types[u], topo.mol[u]);
                if (!site) user2arow[u] = dst;
            }
            continue;
        }
        for (int base = 0; base < len; base += kWave) {
            const int t = base + lane;
            if (t < len) {
                const int u = g.user_unsorted[b + t];
                int r = 0;
                for (int k = 0; k < len; ++k) r += g.user_unsorted[b + k] < u;
                const int dst = b + r;
                g.user[dst] = u;
                g.pos[dst] = wpos[u];
                g.meta[dst] = make_int2(topo.types[u], topo.mol[u]);
                if (!site) user2arow[u] = dst;
            }
        }
    }
}

// Neighbour lists: one block per home cell (atom-grid cells first, then
// site-grid cells).  Rows are padded to the grid's capacity; the true count
// is stored even when it exceeds the capacity, so the host can regrow.
__global__ __launch_bounds__(kListBlock) void k_lists(const GridDev* __restrict__ grids,
                                                      int ncell_a, TopoDev topo,
                                                      double Lx, double Ly, double Lz,
                                                      const int* __restrict__ user2arow,
                                                      int4* __restrict__ a_rec,
                                                      int4* __restrict__ s_rec,
                                                      Status* __restrict__ st)
{
    __shared__ double4 c_pos[kChunk];
    __shared__ int2 c_meta[kChunk];
    __shared__ int c_user[kChunk];
    __shared__ int cell_start[27], cell_cnt[27], cell_pre[28];
    __shared__ int ncells_sh;
    __shared__ int home_cnt[kHomeMax];
    __shared__ int blk_max;
    __shared__ unsigned long long blk_sum;

    const bool site = (int)blockIdx.x >= ncell_a;
    const GridDev& g = grids[site ? 1 : 0];
    const int c = site ? (int)blockIdx.x - ncell_a : (int)blockIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;

    if (threadIdx.x < 27) {
        // one lane per stencil cell: deduplicated offsets, neighbour rank, range
        const int t = threadIdx.x;
        const int ix = t / 9, iy = (t / 3) % 3, iz = t % 3;
        const bool used = ix < g.noff[0] && iy < g.noff[1] && iz < g.noff[2];
        int cnt = 0, s0 = 0;
        if (used) {
            const int lin = g.lin_of_rank[c];
            const int cz = lin % g.n[2];
            const int cy = (lin / g.n[2]) % g.n[1];
            const int cx = lin / (g.n[1] * g.n[2]);
            const int nx = (cx + g.off[0][ix] + g.n[0]) % g.n[0];
            const int ny = (cy + g.off[1][iy] + g.n[1]) % g.n[1];
            const int nz = (cz + g.off[2][iz] + g.n[2]) % g.n[2];
            const int r = g.rank_of_lin[(nx * g.n[1] + ny) * g.n[2] + nz];
            s0 = g.start[r];
            cnt = g.start[r + 1] - s0;
        }
        cell_start[t] = s0;
        cell_cnt[t] = used ? cnt : -1;
    }
    if (threadIdx.x == 0) {
        blk_max = 0;
        blk_sum = 0ull;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int k = 0, acc = 0;
        for (int t = 0; t < 27; ++t) {
            if (cell_cnt[t] < 0) continue;
            cell_start[k] = cell_start[t];
            cell_pre[k] = acc;
            acc += cell_cnt[t];
            ++k;
        }
        cell_pre[k] = acc;
        ncells_sh = k;
    }
    __syncthreads();
    const int ncells = ncells_sh;
    const int ncand = cell_pre[ncells];
    const int hb = g.start[c];
    const int he = g.start[c + 1];
    const double hx = 0.5 * Lx, hy = 0.5 * Ly, hz = 0.5 * Lz;
    const double rl2 = g.rl2;
    const int cap = g.cap;

    for (int hg = hb; hg < he; hg += kHomeMax) {
        const int nh = min(kHomeMax, he - hg);
        for (int h = threadIdx.x; h < nh; h += blockDim.x) home_cnt[h] = 0;
        for (int cb = 0; cb < ncand; cb += kChunk) {
            const int clen = min(kChunk, ncand - cb);
            __syncthreads();
            for (int t = threadIdx.x; t < clen; t += blockDim.x) {
                const int q = cb + t;
                int k = 0;
                while (k + 1 < ncells && cell_pre[k + 1] <= q) ++k;
                const int src = cell_start[k] + (q - cell_pre[k]);
                c_pos[t] = g.pos[src];
                c_meta[t] = g.meta[src];
                c_user[t] = g.user[src];
            }
            __syncthreads();
            for (int h = wave; h < nh; h += nw) {
                const int row = hg + h;
                const double4 pi = g.pos[row];
                const int2 mi = g.meta[row];
                const int ui = g.user[row];
                int eb = 0, ee = 0;
                if (topo.excl_off) {
                    eb = topo.excl_off[ui];
                    ee = topo.excl_off[ui + 1];
                }
                int cnt = home_cnt[h];
                int* out = g.list + (size_t)row * cap;
                for (int base = 0; base < clen; base += kWave) {
                    const int t = base + lane;
                    bool keep = false;
                    uint32_t entry = 0u;
                    if (t < clen) {
                        const int uj = c_user[t];
                        const int2 mj = c_meta[t];
                        keep = uj != ui && !(topo.same_mol && mj.y == mi.y);
                        for (int k = eb; k < ee; ++k)
                            if (topo.excl_idx[k] == uj) keep = false;
                        if (keep) keep = member(pi, c_pos[t], Lx, Ly, Lz, hx, hy, hz, rl2);
                        entry = (uint32_t)uj | ((uint32_t)mj.x << kIdxBits);
                    }
                    const uint64_t mask = __ballot(keep);
                    if (keep) {
                        const int p = cnt + lanes_below(mask);
                        if (p < cap) out[p] = (int)entry;
                    }
                    cnt += __popcll(mask);
                }
                if (lane == 0) home_cnt[h] = cnt;
            }
        }
        __syncthreads();
        for (int h = threadIdx.x; h < nh; h += blockDim.x) {
            const int row = hg + h;
            const int cnt = home_cnt[h];
            g.nrow[row] = cnt;
            atomicMax(&blk_max, cnt);
            atomicAdd(&blk_sum, (unsigned long long)cnt);
            // packed row record for the force kernel: one load per row
            const int u = g.user[row];
            const int ty = g.meta[row].x;
            const int stored = min(cnt, cap);
            if (site) s_rec[row] = make_int4(u, ty, stored, user2arow[u]);
            else a_rec[row] = make_int4(u, ty, stored, topo.hybrid[ty]);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && he > hb) {
        const int slot = blockIdx.x % kStatSlots;
        atomicMax(&st->max_row[site ? 1 : 0][slot], blk_max);
        atomicAdd(&st->entries[site ? 1 : 0][slot], blk_sum);
    }
}

// ---------------------------------------------------------------------------
// force kernel
// ---------------------------------------------------------------------------

template <typename S> __device__ __forceinline__ S rcp(S x);
template <> __device__ __forceinline__ float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double rcp<double>(double x) { return 1.0 / x; }
template <typename S> __device__ __forceinline__ S sqrt_(S x);
template <> __device__ __forceinline__ float sqrt_<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <> __device__ __forceinline__ double sqrt_<double>(double x) { return sqrt(x); }

// Pair terms of the FG part of Eq. 20 (r < r_s+): fpair = -u~'(r)/r and the
// energy.  Called only for r2 < r_s+^2.
template <typename T>
__device__ __forceinline__ void fg_term(const PairCoef<T>& c, const Cutoffs<T>& cut, T r2,
                                        T& fpair, T& en)
{
    if (r2 < cut.rsi2) {
        const T r2i = rcp<T>(r2);
        const T r6i = r2i * r2i * r2i;
        fpair = r6i * (c.fg_c12 * r6i - c.fg_c6) * r2i;
        en = r6i * (c.fg_e12 * r6i - c.fg_e6) - c.fg_shift;
    } else {
        const T r = sqrt_<T>(r2);
        const T d = r - cut.rsi;
        const T dp = c.fg_g[1] + d * (T(2) * c.fg_g[2] + d * (T(3) * c.fg_g[3] + d * (T(4) * c.fg_g[4])));
        fpair = -dp * rcp<T>(r);
        en = c.fg_g[0] + d * (c.fg_g[1] + d * (c.fg_g[2] + d * (c.fg_g[3] + d * c.fg_g[4]))) - c.fg_shift;
    }
}

// Pair terms of the CG part of Eq. 20 (hybrid pairs, r < r_c+).
template <typename T>
__device__ __forceinline__ void cg_term(const PairCoef<T>& c, const Cutoffs<T>& cut, T r2,
                                        T& fpair, T& en)
{
    if (r2 < cut.rsi2) {
        fpair = T(0);
        en = c.sp_g0 - c.cm_shift;
    } else if (r2 < cut.rso2) {
        const T r = sqrt_<T>(r2);
        const T d = r - cut.rsi;
        const T dp = d * d * (T(3) * c.sp_g3 + T(4) * c.sp_g4 * d);
        fpair = -dp * rcp<T>(r);
        en = c.sp_g0 + d * d * d * (c.sp_g3 + d * c.sp_g4) - c.cm_shift;
    } else if (r2 < cut.rci2) {
        const T r2i = rcp<T>(r2);
        const T r6i = r2i * r2i * r2i;
        fpair = r6i * (c.cg_c12 * r6i - c.cg_c6) * r2i;
        en = r6i * (c.cg_e12 * r6i - c.cg_e6) - c.cm_shift;
    } else {
        const T r = sqrt_<T>(r2);
        const T d = r - cut.rci;
        const T dp = c.cm_g[1] + d * (T(2) * c.cm_g[2] + d * (T(3) * c.cm_g[3] + d * (T(4) * c.cm_g[4])));
        fpair = -dp * rcp<T>(r);
        en = c.cm_g[0] + d * (c.cm_g[1] + d * (c.cm_g[2] + d * (c.cm_g[3] + d * c.cm_g[4]))) - c.cm_shift;
    }
}

// Coefficient table staged in LDS when it is small (ntypes <= kLdsTypes).
constexpr int kLdsTypes = 8;

template <typename S, bool EW>
struct CoefLds {
    PairCoef<S> c[kLdsTypes * kLdsTypes];
    PairCoef<double> c64[(EW && sizeof(S) != sizeof(double)) ? kLdsTypes * kLdsTypes : 1];
};

template <typename T>
__device__ __forceinline__ void stage_table(T* dst, const T* __restrict__ src, int count)
{
    const int words = count * (int)(sizeof(T) / sizeof(uint32_t));
    const uint32_t* s = reinterpret_cast<const uint32_t*>(src);
    uint32_t* d = reinterpret_cast<uint32_t*>(dst);
    for (int k = threadIdx.x; k < words; k += blockDim.x) d[k] = s[k];
}

// Entries handled per lane per batch: their list loads, then their position
// gathers, are issued together before any pair term is computed.
constexpr int kBatch = 2;

// One list row: the FG part (CG = false, atom list, zero beyond r_s+) or the
// CG part (CG = true, site list, zero beyond r_c+) of Eq. 20 for every entry.
// Differences are taken in FP64 with the minimum image; the force terms are
// evaluated in S and accumulated in TF; energy and virial terms are always
// evaluated in FP64 (re-evaluated when S is float) and accumulated in FP64.
template <bool CG, typename S, typename TF, bool EW>
__device__ __forceinline__ void row_terms(const ForceArgs& a, const PairCoef<S>* crow,
                                          const PairCoef<double>* crow64,
                                          const Cutoffs<S>& cut, const Cutoffs<double>& cut64,
                                          double xi, double yi, double zi,
                                          const int* __restrict__ lst, int cnt, int sub, int G,
                                          TF& fx, TF& fy, TF& fz, double* acc)
{
    const double rmax2 = CG ? cut64.rco2 : cut64.rso2;
    for (int base = sub; base < cnt; base += G * kBatch) {
        uint32_t e[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int k = base + u * G;
            e[u] = k < cnt ? (uint32_t)lst[k] : 0xffffffffu;
        }
        double px[kBatch], py[kBatch], pz[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int uj = e[u] != 0xffffffffu ? (int)(e[u] & kIdxMask) : 0;
            px[u] = a.pos[3 * uj];
            py[u] = a.pos[3 * uj + 1];
            pz[u] = a.pos[3 * uj + 2];
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            if (e[u] == 0xffffffffu) continue;
            const int tj = (int)(e[u] >> kIdxBits);
            double dx = xi - px[u];
            double dy = yi - py[u];
            double dz = zi - pz[u];
            dx -= a.box[0] * rint(dx * a.inv_box[0]);
            dy -= a.box[1] * rint(dy * a.inv_box[1]);
            dz -= a.box[2] * rint(dz * a.inv_box[2]);
            const double r2d = dx * dx + dy * dy + dz * dz;
            if (r2d < rmax2) {
                S fp, en;
                if constexpr (CG) cg_term<S>(crow[tj], cut, (S)r2d, fp, en);
                else fg_term<S>(crow[tj], cut, (S)r2d, fp, en);
                fx += (TF)(fp * (S)dx);
                fy += (TF)(fp * (S)dy);
                fz += (TF)(fp * (S)dz);
                if constexpr (EW) {
                    double fpd, end;
                    if constexpr (sizeof(S) == sizeof(double)) {
                        fpd = (double)fp;
                        end = (double)en;
                    } else if constexpr (CG) {
                        cg_term<double>(crow64[tj], cut64, r2d, fpd, end);
                    } else {
                        fg_term<double>(crow64[tj], cut64, r2d, fpd, end);
                    }
                    const double hf = 0.5 * fpd;
                    acc[CG ? 1 : 0] += 0.5 * end;
                    acc[2] += hf * dx * dx;
                    acc[3] += hf * dy * dy;
                    acc[4] += hf * dz * dz;
                    acc[5] += hf * dx * dy;
                    acc[6] += hf * dx * dz;
                    acc[7] += hf * dy * dz;
                }
            }
        }
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <typename S, typename TF, bool EW, bool LDS>
__global__ __launch_bounds__(kForceBlock) void k_forces(ForceArgs a, Cutoffs<S> cut,
                                                       Cutoffs<double> cut64)
{
    const bool rb = (int)blockIdx.x >= a.blocks_a;
    const int lb = rb ? (int)blockIdx.x - a.blocks_a : (int)blockIdx.x;
    const int nb = rb ? a.blocks_b : a.blocks_a;
    // Consecutive workgroups are dealt round-robin to the 8 XCDs; give each XCD
    // a contiguous run of rows (neighbouring cells) so they share its L2.
    const int per = nb >> 3;
    const int logical = (lb & 7) * per + (lb >> 3);
    const int lg = rb ? a.log_lanes_b : a.log_lanes_a;
    const int G = 1 << lg;
    const int row = logical * (kForceBlock >> lg) + ((int)threadIdx.x >> lg);
    const int sub = (int)threadIdx.x & (G - 1);

    // row record first: it is the head of every dependent load chain
    int4 rec = make_int4(-1, 0, 0, 1);
    int cnt_a = 0;
    if (!rb) {
        if (row < a.n_arow) rec = a.a_rec[row];
    } else if (row < a.n_srow) {
        rec = a.s_rec[row];
        cnt_a = a.a_rec[rec.w].z;
    }

    const PairCoef<S>* coef;
    const PairCoef<double>* coef64;
    if constexpr (LDS) {
        __shared__ CoefLds<S, EW> tab;
        const int np = a.ntypes * a.ntypes;
        stage_table(tab.c, (const PairCoef<S>*)(sizeof(S) == 8 ? a.coef64 : a.coef32), np);
        if constexpr (EW && sizeof(S) != sizeof(double))
            stage_table(tab.c64, (const PairCoef<double>*)a.coef64, np);
        __syncthreads();
        coef = tab.c;
        if constexpr (EW && sizeof(S) != sizeof(double)) coef64 = tab.c64;
        else coef64 = (const PairCoef<double>*)tab.c;
    } else {
        coef = (const PairCoef<S>*)(sizeof(S) == 8 ? a.coef64 : a.coef32);
        coef64 = (const PairCoef<double>*)a.coef64;
    }

    TF fx = TF(0), fy = TF(0), fz = TF(0);
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const bool own = rb ? rec.x >= 0 : (rec.x >= 0 && rec.w == 0);   // hybrid atom rows belong to the site range
    if (own) {
        const int ui = rec.x, ti = rec.y;
        const double xi = a.pos[3 * ui], yi = a.pos[3 * ui + 1], zi = a.pos[3 * ui + 2];
        const int ar = rb ? rec.w : row;
        const int ca = rb ? cnt_a : rec.z;
        row_terms<false, S, TF, EW>(a, coef + ti * a.ntypes, coef64 + ti * a.ntypes, cut, cut64,
                                    xi, yi, zi, a.a_list + (size_t)ar * a.a_cap, ca, sub, G,
                                    fx, fy, fz, acc);
        if (rb)
            row_terms<true, S, TF, EW>(a, coef + ti * a.ntypes, coef64 + ti * a.ntypes, cut, cut64,
                                       xi, yi, zi, a.s_list + (size_t)row * a.s_cap, rec.z, sub,
                                       G, fx, fy, fz, acc);
    }
    for (int o = G >> 1; o > 0; o >>= 1) {
        fx += __shfl_xor(fx, o);
        fy += __shfl_xor(fy, o);
        fz += __shfl_xor(fz, o);
    }
    if (own && sub == 0) {
        TF* F = (TF*)a.forces;
        F[3 * rec.x] = fx;
        F[3 * rec.x + 1] = fy;
        F[3 * rec.x + 2] = fz;
    }
    if constexpr (EW) {
        // per-block partial sums in a fixed order; k_reduce_ew adds the blocks
        __shared__ double red[8][kForceBlock / kWave];
        const int lane = threadIdx.x & (kWave - 1);
        const int wave = threadIdx.x / kWave;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const double v = wave_sum(acc[k]);
            if (lane == 0) red[k][wave] = v;
        }
        __syncthreads();
        if (threadIdx.x < 8) {
            double t = 0.0;
            for (int w = 0; w < kForceBlock / kWave; ++w) t += red[threadIdx.x][w];
            a.partials[(size_t)blockIdx.x * 8 + threadIdx.x] = t;
        }
    }
}

// Sum of the per-block partials in block order: energy {FG+CG, FG, CG} and the
// six virial components.  One block; deterministic.
__global__ __launch_bounds__(256) void k_reduce_ew(const double* __restrict__ partials, int blocks,
                                                   double* __restrict__ energy,
                                                   double* __restrict__ virial)
{
    __shared__ double red[8][256 / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < blocks; b += blockDim.x)
#pragma unroll
        for (int k = 0; k < 8; ++k) s[k] += partials[(size_t)b * 8 + k];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double v = wave_sum(s[k]);
        if (lane == 0) red[k][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[8];
        for (int k = 0; k < 8; ++k) {
            t[k] = 0.0;
            for (int w = 0; w < 256 / kWave; ++w) t[k] += red[k][w];
        }
        if (energy) {
            energy[0] = t[0] + t[1];
            energy[1] = t[0];
            energy[2] = t[1];
        }
        if (virial)
            for (int k = 0; k < 6; ++k) virial[k] = t[2 + k];
    }
}

__global__ void k_zero_outputs(double* energy, double* virial)
{
    const int t = threadIdx.x;
    if (energy && t < 3) energy[t] = 0.0;
    if (virial && t < 6) virial[t] = 0.0;
}

template <typename S>
Cutoffs<S> cut_as(const double* c64)
{
    Cutoffs<S> c;
    c.rsi = (S)c64[0]; c.rso = (S)c64[1]; c.rci = (S)c64[2]; c.rco = (S)c64[3];
    c.rsi2 = (S)c64[4]; c.rso2 = (S)c64[5]; c.rci2 = (S)c64[6]; c.rco2 = (S)c64[7];
    return c;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

hipError_t launch_bin(int n, const double* pos, const double box[3], TopoDev topo,
                      GridDev* grids_dev, double4* wpos, int2* key_a, int2* key_s, Status* st,
                      hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bin, dim3((n + 255) / 256), dim3(256), 0, s, n, pos, box[0], box[1],
                       box[2], topo, grids_dev, wpos, key_a, key_s, st);
    return hipGetLastError();
}

hipError_t launch_scan(GridDev* grids_dev, int ngrids, Status* st, hipStream_t s)
{
    hipLaunchKernelGGL(k_scan, dim3(ngrids), dim3(kScanThreads), 0, s, grids_dev, st);
    return hipGetLastError();
}

hipError_t launch_scatter(int n, GridDev* grids_dev, const int2* key_a, const int2* key_s,
                          hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3((n + 255) / 256), dim3(256), 0, s, n, grids_dev, key_a,
                       key_s);
    return hipGetLastError();
}

hipError_t launch_cellsort(GridDev* grids_dev, int ncell_a, int ncell_total, const double4* wpos,
                           TopoDev topo, int* user2arow, hipStream_t s)
{
    const int waves_per_block = 4;
    int blocks = (ncell_total + waves_per_block - 1) / waves_per_block;
    if (blocks > 65535) blocks = 65535;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_cellsort, dim3(blocks), dim3(64 * waves_per_block), 0, s, grids_dev,
                       ncell_a, ncell_total, wpos, topo, user2arow);
    return hipGetLastError();
}

hipError_t launch_lists(GridDev* grids_dev, int ncell_a, int ncell_s, TopoDev topo,
                        const double box[3], const int* user2arow, int4* a_rec, int4* s_rec,
                        Status* st, hipStream_t s)
{
    hipLaunchKernelGGL(k_lists, dim3(ncell_a + ncell_s), dim3(kListBlock), 0, s, grids_dev,
                       ncell_a, topo, box[0], box[1], box[2], user2arow, a_rec, s_rec, st);
    return hipGetLastError();
}

hipError_t launch_forces(const ForceArgs& a, const double* cut64, int pair_math, int precision,
                         bool ew, hipStream_t s)
{
    const dim3 grid(a.blocks_a + a.blocks_b), block(kForceBlock);
    const bool lds = a.ntypes <= kLdsTypes;
#define RELRES_LAUNCH(S, TF, EW)                                                                 \
    do {                                                                                         \
        if (lds)                                                                                 \
            hipLaunchKernelGGL((k_forces<S, TF, EW, true>), grid, block, 0, s, a,                \
                               cut_as<S>(cut64), cut_as<double>(cut64));                         \
        else                                                                                     \
            hipLaunchKernelGGL((k_forces<S, TF, EW, false>), grid, block, 0, s, a,               \
                               cut_as<S>(cut64), cut_as<double>(cut64));                         \
    } while (0)
    if (precision == 64) {
        if (ew) RELRES_LAUNCH(double, double, true); else RELRES_LAUNCH(double, double, false);
    } else if (pair_math == 64) {
        if (ew) RELRES_LAUNCH(double, float, true); else RELRES_LAUNCH(double, float, false);
    } else {
        if (ew) RELRES_LAUNCH(float, float, true); else RELRES_LAUNCH(float, float, false);
    }
#undef RELRES_LAUNCH
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !ew) return e;
    hipLaunchKernelGGL(k_reduce_ew, dim3(1), dim3(256), 0, s, a.partials,
                       a.blocks_a + a.blocks_b, a.energy, a.virial);
    return hipGetLastError();
}

hipError_t launch_zero_outputs(double* energy, double* virial, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_outputs, dim3(1), dim3(64), 0, s, energy, virial);
    return hipGetLastError();
}

}  // namespace relres

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
#include "relres_pair.h"
#include "relres_lanes.h"

#include <cstdlib>

namespace relres {
namespace {

constexpr int kWave = 64;
constexpr int kChunk = 256;    // candidates staged in LDS per pass

// Pointers read from the grid descriptors live in device memory, so the
// compiler cannot tell they are global and would use flat instructions, which
// may alias LDS and make every LDS access wait for outstanding global stores.
// Casting them to the global address space gives plain global loads/stores.
#define RELRES_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ RELRES_GLOBAL T* gbl(T* p) { return (RELRES_GLOBAL T*)p; }
// HIP vector types cannot be copied through such pointers; read them as scalars.
// A cell-sorted member carries its list entry and molecule in the fourth
// component of its position: the low 32 bits are the entry (caller index |
// type << kIdxBits), the high 32 bits the molecule.  One 32-byte read gives
// everything the list kernel needs of a member.
__device__ __forceinline__ double member_tag(int u, int type, int mol)
{
    const uint32_t entry = (uint32_t)u | ((uint32_t)type << kIdxBits);
    return __longlong_as_double((long long)(((uint64_t)(uint32_t)mol << 32) | entry));
}
__device__ __forceinline__ void load_member(const double4* base, int i, double& x, double& y,
                                            double& z, uint32_t& entry, int& mol)
{
    RELRES_GLOBAL const double* p = (RELRES_GLOBAL const double*)base + 4 * (size_t)i;
    x = p[0];
    y = p[1];
    z = p[2];
    const uint64_t w = (uint64_t)__double_as_longlong(p[3]);
    entry = (uint32_t)w;
    mol = (int)(uint32_t)(w >> 32);
}
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
// The shift is chosen by selects, not branches: d + (-L) rounds exactly as
// d - L, and adding 0 leaves d (a -0 becomes +0, which squares the same).
__device__ __forceinline__ double min_image(double d, double L, double h)
{
#pragma clang fp contract(off)
    const double s = d > h ? -L : (d < -h ? L : 0.0);
    return d + s;
}

__device__ __forceinline__ bool member(const double4 a, const double4 b, double Lx, double Ly,
                                       double Lz, double hx, double hy, double hz, double rl2)
{
#pragma clang fp contract(off)
    const double dx = min_image(b.x - a.x, Lx, hx);
    const double dy = min_image(b.y - a.y, Ly, hy);
    const double dz = min_image(b.z - a.z, Lz, hz);
    const double r2 = (dx * dx + dy * dy) + dz * dz;
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

// Minimum-image squared distance of (x, y, z) from a wrapped position.
__device__ __forceinline__ double image_dist2(double x, double y, double z, double4 w,
                                              const double* L)
{
    double dx = x - w.x, dy = y - w.y, dz = z - w.z;
    dx -= L[0] * rint(dx / L[0]);
    dy -= L[1] * rint(dy / L[1]);
    dz -= L[2] * rint(dz / L[2]);
    return dx * dx + dy * dy + dz * dz;
}

// Add the lanes of the wave with `flag` set to *count (one atomic per wave).
__device__ __forceinline__ void count_wave(bool flag, unsigned* count)
{
    const unsigned long long m = __ballot(flag);
    if (m != 0ull && (int)(threadIdx.x & (kWave - 1)) == __ffsll((long long)m) - 1)
        atomicAdd(count, (unsigned)__popcll(m));
}

// A slot in cell r of `count` for every lane with `want` set.  Lanes of the
// wave that share a cell take consecutive slots after one atomic add by the
// first of them, so a cell sees one atomic per wave rather than one per atom
// (same-address atomics serialise).  Slot order within a cell is arbitrary;
// the cell sort orders members by caller index afterwards.
__device__ __forceinline__ int claim_slot(int* count, int r, bool want)
{
    const int lane = threadIdx.x & (kWave - 1);
    uint64_t todo = __ballot(want);
    int lead = 0, rank = 0, n_lead = 0;
    while (todo != 0ull) {
        const int l = __ffsll((long long)todo) - 1;
        const int rl = __builtin_amdgcn_readlane(r, l);
        const uint64_t grp = todo & __ballot(r == rl);
        if ((grp >> lane) & 1ull) {
            lead = l;
            rank = __popcll(grp & ((1ull << lane) - 1ull));
        }
        if (lane == l) n_lead = __popcll(grp);
        todo &= ~grp;
    }
    // one atomic instruction for all the groups (their cells are distinct)
    int got = 0;
    if (n_lead > 0) got = atomicAdd(&count[r], n_lead);
    return __shfl(got, lead) + rank;
}

__global__ void k_bin(int n, const double* __restrict__ pos, TopoDev topo,
                      const GridDev* __restrict__ grids, double4* __restrict__ wpos,
                      int2* __restrict__ key_a, int2* __restrict__ key_s, Status* __restrict__ st,
                      int check_moved)
{
    // every lane takes part in the wave's slot claims; lanes past n only vote
    const int i0 = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = i0 < n;
    const int i = in ? i0 : n - 1;
    const int sy = topo.sys ? topo.sys[i] : 0;
    double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    if (!(isfinite(x) && isfinite(y) && isfinite(z))) {
        atomicOr(&st->nonfinite, 1);
        x = y = z = 0.0;
    }
    const GridDev& ga = grids[0];
    const GeomDev& G = ga.geom[sy];
    if (check_moved)   // displacement since the previous build (same boxes and skins)
        count_wave(in && image_dist2(x, y, z, wpos[i], G.box) > G.half_skin2, &st->moved);
    const double wx = wrap_coord(x, G.box[0]), wy = wrap_coord(y, G.box[1]),
                 wz = wrap_coord(z, G.box[2]);
    if (in) wpos[i] = make_double4(wx, wy, wz, 0.0);
    // both grids' cell ranks are read before either slot is claimed
    const int lin = (cell_coord(wx, G.inv_cell[0], G.n[0]) * G.n[1] +
                     cell_coord(wy, G.inv_cell[1], G.n[1])) * G.n[2] +
                    cell_coord(wz, G.inv_cell[2], G.n[2]);
    const int r = gbl(ga.rank_of_lin)[G.cell_base + lin];
    const bool hyb = in && topo.hybrid[topo.types[i]] != 0;
    int rs = -1;
    if (hyb) {
        const GridDev& gs = grids[1];
        const GeomDev& H = gs.geom[sy];
        const int lin_s = (cell_coord(wx, H.inv_cell[0], H.n[0]) * H.n[1] +
                           cell_coord(wy, H.inv_cell[1], H.n[1])) * H.n[2] +
                          cell_coord(wz, H.inv_cell[2], H.n[2]);
        rs = gbl(gs.rank_of_lin)[H.cell_base + lin_s];
    }
    {
        const int slot = claim_slot(ga.count, r, in);
        if (in) key_a[i] = make_int2(r, slot);
        // one-launch placement: the member goes straight into its cell's bucket
        if (in && slot < ga.bucket_cap)
            gbl(ga.user_unsorted)[(size_t)r * ga.bucket_cap + slot] = i;
    }
    // grids[1] is grids[0] again when there are no sites (no hybrid lanes then)
    const int slot_s = claim_slot(grids[1].count, rs, hyb);
    if (in) key_s[i] = hyb ? make_int2(rs, slot_s) : make_int2(-1, -1);
    if (hyb && slot_s < grids[1].bucket_cap)
        gbl(grids[1].user_unsorted)[(size_t)rs * grids[1].bucket_cap + slot_s] = i;
}

// Atoms now more than half the skin from their position at the last build.
__global__ void k_moved(int n, const double* __restrict__ pos, TopoDev topo,
                        const GridDev* __restrict__ grids, const double4* __restrict__ wpos,
                        Status* __restrict__ st)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int sy = topo.sys ? topo.sys[i] : 0;
    const double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    const GeomDev& G = grids[0].geom[sy];
    // a non-finite position counts as moved (the comparison is false for NaN)
    count_wave(!(image_dist2(x, y, z, wpos[i], G.box) <= G.half_skin2), &st->moved_query);
}

// One block per grid: exclusive scan of the per-cell counts into `start`,
// then the counts are cleared for the next build.  Counts are staged through
// LDS in segments of kScanSeg cells with coalesced loads; each thread scans a
// contiguous run of its segment.  Block 0 also clears the list statistics.
constexpr int kScanThreads = 1024;
constexpr int kScanSeg = 8192;

// Exclusive prefix sum over the block of one int per thread (in thread
// order); every thread also gets the block's total.  Each wave scans its
// lanes with cross-lane shuffles, then adds the totals of the waves before
// it: two block barriers in all.
__device__ __forceinline__ int block_exclusive_scan(int v, int* wtot, int& total)
{
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wtot[w] = x;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / kWave; ++k) {
        const int t = wtot[k];
        before += k < w ? t : 0;
        all += t;
    }
    __syncthreads();            // wtot is reused by the next call
    total = all;
    return before + x - v;
}

// One segment of the scan (all threads of the block): start[seg + k] =
// carry + the exclusive prefix of the segment's counts, the counts cleared.
// Returns the segment's total in every thread.
__device__ __forceinline__ int scan_segment(int* vals, int* sums, RELRES_GLOBAL int* gcount,
                                            RELRES_GLOBAL int* gstart, int seg, int len, int carry)
{
    const int t = threadIdx.x;
    constexpr int per = kScanSeg / kScanThreads;
    for (int k = t; k < kScanSeg; k += kScanThreads) vals[k] = k < len ? gcount[seg + k] : 0;
    __syncthreads();
    int s = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) s += vals[t * per + k];
    int total;
    int run = carry + block_exclusive_scan(s, sums, total);
#pragma unroll
    for (int k = 0; k < per; ++k) {
        const int v = vals[t * per + k];
        vals[t * per + k] = run;
        run += v;
    }
    __syncthreads();
    for (int k = t; k < len; k += kScanThreads) {
        gstart[seg + k] = vals[k];
        gcount[seg + k] = 0;
    }
    __syncthreads();            // vals is reused by the next segment
    return total;
}

// Sum of one int per thread over the block (every thread gets it).
__device__ __forceinline__ int block_sum_int(int v, int* sums)
{
    int total;
    block_exclusive_scan(v, sums, total);
    return total;
}

// One block per grid: exclusive scan of the per-cell counts into `start`,
// then the counts are cleared for the next build.  Counts are staged through
// LDS in segments of kScanSeg cells with coalesced loads; each thread scans a
// contiguous run of its segment.
__global__ __launch_bounds__(kScanThreads) void k_scan(GridDev* __restrict__ grids)
{
    __shared__ int vals[kScanSeg];
    __shared__ int sums[kScanThreads];
    const GridDev& g = grids[blockIdx.x];
    const int nc = g.ncell;
    int carry = 0;
    for (int seg = 0; seg < nc; seg += kScanSeg)
        carry += scan_segment(vals, sums, gbl(g.count), gbl(g.start), seg, min(kScanSeg, nc - seg),
                              carry);
    if (threadIdx.x == 0) gbl(g.start)[nc] = carry;
}

// Grids of more than one segment: the same scan with every segment in a
// block of its own.  Blocks 0 .. nseg0-1 are the segments of grid 0, the
// rest those of grid 1.  First each block sums its segment's counts ...
__global__ __launch_bounds__(kScanThreads) void k_scan_totals(const GridDev* __restrict__ grids,
                                                              int nseg0, int* __restrict__ seg_tot)
{
    __shared__ int sums[kScanThreads];
    const int b = blockIdx.x;
    const int gi = b >= nseg0 ? 1 : 0;
    const int seg = (gi ? b - nseg0 : b) * kScanSeg;
    const GridDev& g = grids[gi];
    const int len = min(kScanSeg, g.ncell - seg);
    RELRES_GLOBAL const int* gcount = gbl(g.count);
    int s = 0;
    for (int k = threadIdx.x; k < len; k += kScanThreads) s += gcount[seg + k];
    s = block_sum_int(s, sums);
    if (threadIdx.x == 0) seg_tot[b] = s;
}

// ... then each block adds the totals of its grid's earlier segments and
// scans its own segment (the grid's last segment also writes start[ncell]).
__global__ __launch_bounds__(kScanThreads) void k_scan_segments(GridDev* __restrict__ grids,
                                                                int nseg0,
                                                                const int* __restrict__ seg_tot)
{
    __shared__ int vals[kScanSeg];
    __shared__ int sums[kScanThreads];
    const int b = blockIdx.x;
    const int gi = b >= nseg0 ? 1 : 0;
    const int q = gi ? b - nseg0 : b;
    const int first = gi ? nseg0 : 0;
    const GridDev& g = grids[gi];
    const int nc = g.ncell;
    const int seg = q * kScanSeg;
    int carry = 0;
    for (int j = threadIdx.x; j < q; j += kScanThreads) carry += seg_tot[first + j];
    carry = block_sum_int(carry, sums);
    const int len = min(kScanSeg, nc - seg);
    const int total = scan_segment(vals, sums, gbl(g.count), gbl(g.start), seg, len, carry);
    if (threadIdx.x == 0 && seg + len == nc) gbl(g.start)[nc] = carry + total;
}

__global__ void k_scatter(int n, const GridDev* __restrict__ grids, const int2* __restrict__ key_a,
                          const int2* __restrict__ key_s)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int2 ka = key_a[i];
    gbl(grids[0].user_unsorted)[gbl(grids[0].start)[ka.x] + ka.y] = i;
    const int2 ks = key_s[i];
    if (ks.x >= 0) gbl(grids[1].user_unsorted)[gbl(grids[1].start)[ks.x] + ks.y] = i;
}

__device__ __forceinline__ int readlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
// A wave-uniform double moved to scalar registers.
__device__ __forceinline__ double readfirst_d(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double readlane_d(double v, int l)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Cell sort: order the members of every cell by caller index (rank by
// counting) and write the sorted position / (type, molecule) / index / cell
// arrays.  A wave takes kWave / G consecutive cells, one group of G lanes
// each; a cell of at most G members is ranked within its group by cross-lane
// reads, a larger one by the whole wave after the small ones.  G = 16 suits
// grids of a few members per cell, G = 64 (one cell per wave) crowded ones.

__device__ __forceinline__ void place_read(const GridDev& g, bool site, int c, int dst, int u,
                                           double4 p, int ty, int mol,
                                           int* __restrict__ user2arow)
{
    gbl(g.user)[dst] = u;
    g.pos[dst] = make_double4(p.x, p.y, p.z, member_tag(u, ty, mol));   // generic store (no LDS use here)
    g.meta[dst] = make_int2(ty, mol);
    gbl(g.row_cell)[dst] = c;
    if (!site) user2arow[u] = dst;
}

__device__ __forceinline__ void place_member(const GridDev& g, bool site, int c, int dst, int u,
                                             const double4* __restrict__ wpos, const TopoDev& topo,
                                             int* __restrict__ user2arow)
{
    place_read(g, site, c, dst, u, wpos[u], topo.types[u], topo.mol[u], user2arow);
}

template <int kSortGroup>
__global__ void k_cellsort(const GridDev* __restrict__ grids, int ncell_a, int ncell_total,
                           const double4* __restrict__ wpos, TopoDev topo,
                           int* __restrict__ user2arow)
{
    constexpr int kSortCells = kWave / kSortGroup;
    const int lane = threadIdx.x & (kWave - 1);
    const int q = lane / kSortGroup, gl = lane & (kSortGroup - 1);
    const int wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
    const int nwaves = (gridDim.x * blockDim.x) / kWave;
    for (int c0 = wave * kSortCells; c0 < ncell_total; c0 += nwaves * kSortCells) {
        // group q: cell c0 + q (cells past the end are empty)
        const int cell = c0 + q;
        const bool site = cell >= ncell_a;
        const GridDev& g = grids[site ? 1 : 0];
        const int c = site ? cell - ncell_a : cell;
        int b = 0, len = 0;
        if (cell < ncell_total) {
            RELRES_GLOBAL const int* gstart = gbl(g.start);
            b = gstart[c];
            len = gstart[c + 1] - b;
        }
        const bool small = len <= kSortGroup;
        const int u = (small && gl < len) ? gbl(g.user_unsorted)[b + gl] : 0x7fffffff;
        int r = 0;
        if constexpr (kSortGroup < kWave) {
#pragma unroll
            for (int k = 0; k < kSortGroup; ++k)
                r += __shfl(u, (lane & ~(kSortGroup - 1)) + k) < u;
        } else {
            const int m = small ? len : 0;      // one cell per wave: len is uniform
            for (int k = 0; k < m; ++k) r += __shfl(u, k) < u;
        }
        if (small && gl < len) place_member(g, site, c, b + r, u, wpos, topo, user2arow);
        // the larger cells of this wave, one at a time with the whole wave
        for (int k = 0; k < kSortCells; ++k) {
            const int lenk = readlane_i(len, k * kSortGroup);
            if (lenk <= kSortGroup) continue;
            const int cellk = c0 + k;
            const bool sitek = cellk >= ncell_a;
            const GridDev& gk = grids[sitek ? 1 : 0];
            const int ck = sitek ? cellk - ncell_a : cellk;
            const int bk = readlane_i(b, k * kSortGroup);
            RELRES_GLOBAL const int* guu = gbl(gk.user_unsorted);
            if (lenk <= kWave) {
                const int v = lane < lenk ? guu[bk + lane] : 0x7fffffff;
                int rk = 0;
                for (int j = 0; j < lenk; ++j) rk += __shfl(v, j) < v;
                if (lane < lenk) place_member(gk, sitek, ck, bk + rk, v, wpos, topo, user2arow);
                continue;
            }
            for (int base = 0; base < lenk; base += kWave) {
                const int t = base + lane;
                if (t < lenk) {
                    const int v = guu[bk + t];
                    int rk = 0;
                    for (int j = 0; j < lenk; ++j) rk += guu[bk + j] < v;
                    place_member(gk, sitek, ck, bk + rk, v, wpos, topo, user2arow);
                }
            }
        }
    }
}


// Scan, scatter and cell sort in one launch, for grids of few cells whose
// members k_bin has filed into per-cell buckets of bucket_cap slots.  A block
// takes kCells consecutive cells of one grid (the atom grid's blocks first):
// it adds up the counts of every cell before its own (each block repeats
// this, so it suits a few thousand cells), writes its cells' starts, then
// ranks each cell's members by caller index as k_cellsort does and writes
// the sorted arrays.  A cell with more members than its bucket holds finds
// them, already in caller order, by a wave-wide pass over the key array.
// The counts stay as they are: the list kernel clears them.
constexpr int kPlaceThreads = 256;

template <int kSortGroup>
__global__ __launch_bounds__(kPlaceThreads) void k_place(const GridDev* __restrict__ grids,
                                                         int blocks_a, int n,
                                                         const int2* __restrict__ key_a,
                                                         const int2* __restrict__ key_s,
                                                         const double4* __restrict__ wpos,
                                                         TopoDev topo, int* __restrict__ user2arow)
{
    constexpr int kWaves = kPlaceThreads / kWave;
    constexpr int kCellsPerWave = kWave / kSortGroup;
    constexpr int kCells = kWaves * kCellsPerWave;     // at most 64: one wave scans them
    __shared__ int wtot[kWaves];
    __shared__ int cnt_sh[kCells], first_sh[kCells];
    const bool site = (int)blockIdx.x >= blocks_a;
    const GridDev& g = grids[site ? 1 : 0];
    const int c0 = ((int)blockIdx.x - (site ? blocks_a : 0)) * kCells;
    const int nc = g.ncell;
    const int cap = g.bucket_cap;
    RELRES_GLOBAL const int* gcount = gbl(g.count);
    RELRES_GLOBAL int* gstart = gbl(g.start);
    RELRES_GLOBAL const int* bucket = gbl(g.user_unsorted);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    // group q of G lanes: cell c0 + wave * kCellsPerWave + q
    const int q = lane / kSortGroup, gl = lane & (kSortGroup - 1);
    const int ci = wave * kCellsPerWave + q;
    const int c = c0 + ci;
    const int in_group = kSortGroup < cap ? kSortGroup : cap;

    // Every read that does not depend on another is issued first: the
    // block's own counts (wave 0), the first in_group bucket slots of each
    // group's cell (whatever the cell's count; slots past it are dropped
    // below) and the counts of the cells before this block's.
    const int own_cnt = (wave == 0 && lane < kCells && c0 + lane < nc) ? gcount[c0 + lane] : 0;
    const int u_slot = (c < nc && gl < in_group) ? bucket[(size_t)c * cap + gl] : 0x7fffffff;
    // members of the grid's cells before this block's: c0 is a multiple of 4,
    // so the counts are read as int4, four loads per thread in flight at once
    // (the first round outside the loop, so its reads go out with the ones
    // above; grids of more than 4096 cells before the block loop further)
    // (global 16-byte reads of clamped index, the ones past the end dropped,
    // so no branch splits them)
    int s = 0;
    const int n4 = c0 >> 2;
    if (n4 > 0) {
        typedef int int4v __attribute__((ext_vector_type(4)));
        RELRES_GLOBAL const int4v* c4 = (RELRES_GLOBAL const int4v*)gcount;
        auto round = [&](int base) {
            int4v q4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = base + u * kPlaceThreads + (int)threadIdx.x;
                const int4v v = c4[min(k, n4 - 1)];
                q4[u] = k < n4 ? v : (int4v)(0);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) s += (q4[u].x + q4[u].y) + (q4[u].z + q4[u].w);
        };
        round(0);
        for (int base = 4 * kPlaceThreads; base < n4; base += 4 * kPlaceThreads) round(base);
    }
    // the slot's member (position, type, molecule) is read once its index
    // and the counts are in, while the counts are summed and scanned: a slot past its cell's count
    // holds an index of an earlier build (garbage before the first), so only
    // indices below n are read, and such a read is dropped
    const int u_pre = (unsigned)u_slot < (unsigned)n ? u_slot : 0;
    const double4 p_pre = wpos[u_pre];
    const int ty_pre = topo.types[u_pre], mol_pre = topo.mol[u_pre];
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) s += __shfl_xor(s, o);
    if (lane == 0) wtot[wave] = s;
    __syncthreads();
    if (wave == 0) {
        int carry = 0;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) carry += wtot[k];
        const int v = own_cnt;
        int x = v;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane < kCells) {
            cnt_sh[lane] = v;
            first_sh[lane] = carry + x - v;
            if (c0 + lane < nc) gstart[c0 + lane] = carry + x - v;
            if (c0 + lane == nc - 1) gstart[nc] = carry + x;
        }
    }
    __syncthreads();

    const int len = c < nc ? cnt_sh[ci] : 0;
    const int b = first_sh[ci];
    const bool small = len <= in_group;
    const int u = (small && gl < len) ? u_slot : 0x7fffffff;
    int r = 0;
    if constexpr (kSortGroup < kWave) {
#pragma unroll
        for (int k = 0; k < kSortGroup; ++k) r += __shfl(u, (lane & ~(kSortGroup - 1)) + k) < u;
    } else {
        const int m = small ? len : 0;      // one cell per wave: len is uniform
        for (int k = 0; k < m; ++k) r += __shfl(u, k) < u;
    }
    if (small && gl < len) place_read(g, site, c, b + r, u, p_pre, ty_pre, mol_pre, user2arow);
    // the larger cells of this wave, one at a time with the whole wave
    for (int k = 0; k < kCellsPerWave; ++k) {
        const int lenk = readlane_i(len, k * kSortGroup);
        if (lenk <= in_group) continue;
        const int ck = c0 + wave * kCellsPerWave + k;
        const int bk = readlane_i(b, k * kSortGroup);
        if (lenk <= cap) {                  // cap <= 64: one member per lane
            const int v = lane < lenk ? bucket[(size_t)ck * cap + lane] : 0x7fffffff;
            int rk = 0;
            for (int j = 0; j < lenk; ++j) rk += __shfl(v, j) < v;
            if (lane < lenk) place_member(g, site, ck, bk + rk, v, wpos, topo, user2arow);
            continue;
        }
        // the cell outgrew its bucket: its members in caller order from the keys
        const int2* __restrict__ key = site ? key_s : key_a;
        int run = 0;
        for (int i0 = 0; i0 < n; i0 += kWave) {
            const int i = i0 + lane;
            const bool mine = i < n && key[i].x == ck;
            const uint64_t m = __ballot(mine);
            if (mine) place_member(g, site, ck, bk + run + lanes_below(m), i, wpos, topo, user2arow);
            run += __popcll(m);
        }
    }
}

// After a one-launch placement the cell counts are still set: the list
// kernel, the next launch of the build, clears them for the next build (the
// grid array always has two entries; the second repeats the first when there
// are no sites).
__device__ __forceinline__ void clear_bucket_counts(const GridDev* __restrict__ grids)
{
    const int stride = (int)(gridDim.x * blockDim.x);
    for (int gi = 0; gi < 2; ++gi) {
        const GridDev& g = grids[gi];
        if (g.bucket_cap <= 0) continue;
        RELRES_GLOBAL int* cnt = gbl(g.count);
        for (int c = (int)(blockIdx.x * blockDim.x + threadIdx.x); c < g.ncell; c += stride)
            cnt[c] = 0;
    }
}

// Membership with the periodic shift of the candidate's stencil slot known in
// advance.  When a grid has at least four cells along an axis, a neighbour
// cell reached without wrapping lies within two cells (< L/2) of the home
// atom, and one reached by wrapping lies more than L/2 away in the direction
// of the wrap.  The single-shift recipe therefore applies exactly `shift`
// (0 or -+L), and (x_j - x_i) + shift rounds exactly as the recipe's
// (x_j - x_i) followed by "-= L" / "+= L".
__device__ __forceinline__ bool member_shifted(double xi, double yi, double zi, double xj,
                                               double yj, double zj, double sx, double sy,
                                               double sz, double rl2)
{
#pragma clang fp contract(off)
    const double dx = (xj - xi) + sx;
    const double dy = (yj - yi) + sy;
    const double dz = (zj - zi) + sz;
    const double r2 = (dx * dx + dy * dy) + dz * dz;
    return r2 < rl2;
}

constexpr int kResidentListWaves = 256 * 4 * 3;

// A compile-time bool as a value (selects one of two instantiations of a
// generic lambda).
template <bool B>
struct BoolC {
    static constexpr bool value = B;
};

// Stencil geometry: S cells per axis around the home cell (3 for cells of at
// least the list radius, 5 for cells of at least half of it), S^3 slots in
// x-major order, slot tables of kSlotTab entries per wave.
template <int S>
struct Stencil {
    static constexpr int kHalf = S / 2;
    static constexpr int kSlots = S * S * S;
    static constexpr int kTab = S == 3 ? 32 : 128;
    static constexpr int kPerLane = S == 3 ? 1 : 2;   // slots a lane holds: lane, lane + 64
    // the offset of slot s along axis a (0 = x) in cells
    static __device__ __forceinline__ int off(int s, int a)
    {
        const int d = a == 0 ? s / (S * S) : (a == 1 ? (s / S) % S : s % S);
        return d - kHalf;
    }
};

// Global rank of the cell at offset (ox, oy, oz) from the cell (hx, hy, hz)
// of a grid of n cells per axis, or -1 when the offset repeats a cell that a
// smaller offset already reaches (an axis of fewer than S cells keeps its
// first n offsets, which reach every cell once).
template <int S>
__device__ __forceinline__ int stencil_rank(const GeomDev& G, RELRES_GLOBAL const int* grank,
                                            int hx, int hy, int hz, int s)
{
    using St = Stencil<S>;
    if (s >= St::kSlots) return -1;
    const int ox = St::off(s, 0), oy = St::off(s, 1), oz = St::off(s, 2);
    const int n0 = G.n[0], n1 = G.n[1], n2 = G.n[2];
    if ((n0 < S && ox + St::kHalf >= n0) || (n1 < S && oy + St::kHalf >= n1) ||
        (n2 < S && oz + St::kHalf >= n2))
        return -1;
    const int x = (hx + ox + 2 * n0) % n0, y = (hy + oy + 2 * n1) % n1, z = (hz + oz + 2 * n2) % n2;
    return grank[G.cell_base + (x * n1 + y) * n2 + z];
}

// Neighbour lists, one wave per group of R consecutive member rows (rows are
// in cell order, so a group spans one or a few cells).  Work per wave is
// bounded by the group size, so crowded cells are spread over many waves.
// Each lane owns one home row of the group: its position, exclusions and
// running count live in that lane and are broadcast with readlane.  The
// candidates of the home cell's stencil are loaded straight into registers,
// K per lane per round (candidate q in lane q % 64), and every home row of
// the cell tests them there, so a candidate is read from memory once per cell
// and never through LDS.  A larger K takes fewer rounds but more registers:
// it pays when all waves of the launch are resident at once.  Candidates are
// visited in stencil-slot order, each row's entries are appended in that
// order with a wave ballot.  Only wave-level synchronisation is used, so
// waves of one block may run different trip counts.  S is the stencil width
// of the grid the wave's rows belong to (3: cells of one list radius; 5:
// cells of half of it, fewer candidates per row and more cells per wave).
template <int K, int S>
__device__ __forceinline__ void list_wave(const GridDev& g, int wv, int lw, bool site, int max_excl,
                                          const TopoDev& topo, const int* __restrict__ user2arow,
                                          int4* __restrict__ a_rec, int4* __restrict__ s_rec,
                                          Status* __restrict__ st, int* slot_base,
                                          double* slot_shift, int* slot_win,
                                          int* excl_lds)
{
    using St = Stencil<S>;
    const int lane = threadIdx.x & (kWave - 1);
    const double4* gpos = g.pos;      // read through load_member
    RELRES_GLOBAL const int* gstart = gbl(g.start);
    RELRES_GLOBAL const int* gnbr = gbl(g.nbr);
    RELRES_GLOBAL const int* grank = gbl(g.rank_of_lin);
    RELRES_GLOBAL int* glist = gbl(g.list);
    RELRES_GLOBAL const int* glor = gbl(g.lin_of_rank);
    // the system whose grid holds this wave's rows (wave-uniform; grids with
    // no rows have no waves)
    const int gs_lo = g.nsys > 1 ? __builtin_amdgcn_readfirstlane(g.wave_sys[lw]) : 0;
    const GeomDev& G = g.geom[gs_lo];
    // the grid's cell counts are wave-uniform: readfirstlane keeps them (and
    // the cell arithmetic on them) in scalar registers, where the compiler
    // would otherwise hold the values it read in vector registers (the box
    // edges stay there: the selects of the image shifts take them so)
    const int n0 = __builtin_amdgcn_readfirstlane(G.n[0]);
    const int n1 = __builtin_amdgcn_readfirstlane(G.n[1]);
    const int n2 = __builtin_amdgcn_readfirstlane(G.n[2]);
    const double Lx = G.box[0], Ly = G.box[1], Lz = G.box[2];
    // known image shifts: every stencil slot a distinct cell with one
    // periodic image (at least four cells per axis for the 27-cell stencil,
    // five for the 125-cell one)
    // (wave-uniform; readfirstlane makes the choice a scalar branch)
    const bool known_shift = __builtin_amdgcn_readfirstlane(
        S == 3 ? (n0 >= 4 && n1 >= 4 && n2 >= 4) : (n0 >= 5 && n1 >= 5 && n2 >= 5));
    const int R = g.rows_per_wave;
    const int r0 = __builtin_amdgcn_readfirstlane(G.row_base + (lw - G.wave_base) * R);
    const int r1 = __builtin_amdgcn_readfirstlane(min(G.row_base + G.members, r0 + R));
    const double hx = G.half[0], hy = G.half[1], hz = G.half[2];
    const double rl2 = readfirst_d(G.rl2);
    const int cap = g.cap;
    const int* __restrict__ excl_off = topo.excl_off;
    const int* __restrict__ excl_idx = topo.excl_idx;
    const int same_mol = topo.same_mol;
    // exclusion lists of the wave's home rows, staged once (kRowsPerWave x max_excl)
    int* my_excl = excl_lds + wv * kRowsPerWave * max_excl;

    // lane h < (r1 - r0) owns home row r0 + h
    const int nh = r1 - r0;
    const int myrow = r0 + lane;
    double mx = 0.0, my = 0.0, mz = 0.0;
    int mt = 0, mmol = 0;
    int mu = -1, mne = 0, marow = 0, mcell = -1, mcnt = 0;   // mne: exclusions of the row
    if (lane < nh) {
        uint32_t ment;
        load_member(gpos, myrow, mx, my, mz, ment, mmol);
        mu = (int)(ment & kIdxMask);
        mt = (int)(ment >> kIdxBits);
        mcell = gbl(g.row_cell)[myrow];
        if (excl_off) {
            const int meb = excl_off[mu];
            mne = excl_off[mu + 1] - meb;
            for (int k = 0; k < mne; ++k) my_excl[lane * max_excl + k] = excl_idx[meb + k];
        }
        if (site) marow = user2arow[mu];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // The stencil slots a lane holds (slot `lane`, and `lane + 64` for the
    // 125-cell stencil) of a home cell: the slot's cell (rank, or -1), then
    // the first member and the end of its member range.  The next home cell's
    // reads are issued while this cell is processed (the ranks before this
    // cell's first candidate reads, the ranges at its first round), so the
    // dependent reads leave the per-cell critical path.  The range reads are
    // unconditional (lanes past the stencil and empty slots read a valid entry
    // and drop it at use), so no branch makes the compiler wait for them early.
    int next_rank[St::kPerLane];
    int next_lin = 0;      // the next home cell's linear index (its coordinates)
    auto ranks_of = [&](int h) {
        const int c = readlane_i(mcell, h);
        next_lin = glor[c];
        if constexpr (S == 3) {
            next_rank[0] = gnbr[c * 27 + min(lane, 26)];
        } else {
            const int lin = __builtin_amdgcn_readfirstlane(next_lin);
            const int cz = lin % n2, cy = (lin / n2) % n1, cx = lin / (n1 * n2);
#pragma unroll
            for (int u = 0; u < St::kPerLane; ++u)
                next_rank[u] = stencil_rank<S>(G, grank, cx, cy, cz, lane + kWave * u);
        }
    };
    auto no_ranks = [&]() {
#pragma unroll
        for (int u = 0; u < St::kPerLane; ++u) next_rank[u] = -1;
    };
    auto slot_valid = [&](int u) {
        return lane + kWave * u < St::kSlots && next_rank[u] >= 0;
    };
    if (nh > 0) ranks_of(0); else no_ranks();
    int next_lo[St::kPerLane], next_hi[St::kPerLane];
    auto range_of = [&]() {
#pragma unroll
        for (int u = 0; u < St::kPerLane; ++u) {
            int r = next_rank[u];
            // keeps the rank's first use here, after this cell's candidate
            // loads were issued: hoisted ahead of them, it would make the
            // wave wait for the rank read first
            asm volatile("" : "+v"(r));
            r = lane + kWave * u < St::kSlots && r >= 0 ? r : 0;
            next_lo[u] = gstart[r];
            next_hi[u] = gstart[r + 1];
        }
    };
    if (nh > 0) range_of();
    int h0 = 0;
    while (h0 < nh) {
        // rows h0 .. h1-1 share one cell
        const int c = readlane_i(mcell, h0);
        int h1 = h0 + 1;
        while (h1 < nh && readlane_i(mcell, h1) == c) ++h1;
        h1 = __builtin_amdgcn_readfirstlane(h1);   // wave-uniform: a scalar row loop
        int s0[St::kPerLane], cnt[St::kPerLane];
#pragma unroll
        for (int u = 0; u < St::kPerLane; ++u) {
            const bool ok = slot_valid(u);
            s0[u] = ok ? next_lo[u] : 0;
            cnt[u] = ok ? next_hi[u] - next_lo[u] : 0;
        }
        // this cell's linear index, read one cell ahead with its stencil ranks
        const int lin_c = __builtin_amdgcn_readfirstlane(next_lin);
        if (h1 < nh) ranks_of(h1); else no_ranks();
        // home cell coordinates: the periodic shift of every stencil slot
        int cx = 0, cy = 0, cz = 0;
        if (known_shift) {
            cz = lin_c % n2;
            cy = (lin_c / n2) % n1;
            cx = lin_c / (n1 * n2);
        }
        // first candidate of every slot: a wave scan of the counts in slot
        // order (slot lane, then slot lane + 64); with known shifts, each
        // slot's periodic image shift (-L, 0 or +L per axis) is tabulated
        // once here instead of per candidate
        int ncand = 0;
        int first[St::kPerLane];
#pragma unroll
        for (int u = 0; u < St::kPerLane; ++u) {
            const int pre = wave_inclusive_scan(cnt[u]);
            const int slot = lane + kWave * u;
            first[u] = ncand + pre - cnt[u];
            if (slot < St::kTab) {
                // member index of candidate q of this slot: slot_base + q
                slot_base[slot] = s0[u] - first[u];
            }
            if (known_shift && slot < St::kSlots) {
                const int ox = St::off(slot, 0), oy = St::off(slot, 1), oz = St::off(slot, 2);
                slot_shift[slot] = cx + ox < 0 ? -Lx : (cx + ox >= n0 ? Lx : 0.0);
                slot_shift[St::kTab + slot] = cy + oy < 0 ? -Ly : (cy + oy >= n1 ? Ly : 0.0);
                slot_shift[2 * St::kTab + slot] = cz + oz < 0 ? -Lz : (cz + oz >= n2 ? Lz : 0.0);
            }
            ncand += __builtin_amdgcn_readfirstlane(__shfl(pre, kWave - 1));
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        int carry = -1;      // the slot of candidate cb - 1
        for (int cb = 0; cb < ncand; cb += kWave * K) {
            // The slot of each of the round's 64 K candidates (cb + p for p =
            // lane + 64 k): every non-empty slot marks its first candidate in
            // a window of the round (candidate cb + p at (p % 64) K + p / 64,
            // so a lane's K entries are one vector read), and a running
            // maximum in candidate order carries each mark over the slot's
            // other candidates.
#pragma unroll
            for (int k = 0; k < K; ++k) slot_win[lane * K + k] = -1;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int u = 0; u < St::kPerLane; ++u) {
                const int p = first[u] - cb;
                if (cnt[u] > 0 && p >= 0 && p < kWave * K)
                    slot_win[(p & (kWave - 1)) * K + (p >> 6)] = lane + kWave * u;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            int cslot[K];
#pragma unroll
            for (int k = 0; k < K; ++k) cslot[k] = slot_win[lane * K + k];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                cslot[k] = max(wave_inclusive_max(cslot[k]), carry);
                carry = __builtin_amdgcn_readlane(cslot[k], kWave - 1);
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            double px[K], py[K], pz[K];
            uint32_t pe[K];     // the candidate's list entry
            int pm[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int q = cb + lane + kWave * k;
                px[k] = py[k] = pz[k] = 0.0;
                pe[k] = 0;
                pm[k] = 0;
                if (q < ncand)
                    load_member(gpos, slot_base[max(cslot[k], 0)] + q, px[k], py[k], pz[k],
                                pe[k], pm[k]);
            }
            // the next cell's member ranges (its stencil ranks were read at
            // this cell's start), issued after this cell's first candidate
            // reads and once per cell, outside the rows' loop
            if (cb == 0) range_of();
            // periodic image shift of the candidate's slot, taken once per
            // candidate for all the rows
            double sx[K], sy[K], sz[K];
            int pu[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const bool ok = cb + lane + kWave * k < ncand;
                const int slot = max(cslot[k], 0);
                pu[k] = ok ? (int)(pe[k] & kIdxMask) : -1;
                sx[k] = sy[k] = sz[k] = 0.0;
                if (known_shift && ok) {
                    sx[k] = slot_shift[slot];
                    sy[k] = slot_shift[St::kTab + slot];
                    sz[k] = slot_shift[2 * St::kTab + slot];
                }
            }
            // The conditions of a (row, candidate) pair other than the
            // distance are wave lane masks, one per k, combined with scalar
            // ANDs: a lane's own work per row is its compares and its
            // distance test.  `live` marks the slots holding a candidate.
            uint64_t live[K];
#pragma unroll
            for (int k = 0; k < K; ++k) live[k] = __ballot(pu[k] >= 0);
            // The rows' loop, instantiated for known image shifts and for
            // the minimum image by comparison, each with and without the
            // same-molecule exclusion, so each choice is one scalar branch
            // per round and not a select or a branch per test.  Every cell
            // has at least one home row (h1 > h0): a loop that always runs,
            // so no path skips it with candidate reads pending.
            auto row_loop = [&](auto known, auto own_mol) {
            constexpr bool kKnown = decltype(known)::value;
            constexpr bool kSameMol = decltype(own_mol)::value;
            int h = __builtin_amdgcn_readfirstlane(h0);
            do {
                const double xi = readlane_d(mx, h), yi = readlane_d(my, h), zi = readlane_d(mz, h);
                const int ui = readlane_i(mu, h);
                const int moli = readlane_i(mmol, h);
                const int ne = readlane_i(mne, h);
                const int* hex = my_excl + h * max_excl;
                int hc = readlane_i(mcnt, h);
                RELRES_GLOBAL int* out =
                    glist + (size_t)__builtin_amdgcn_readfirstlane(r0 + h) * cap;
                uint64_t keep[K];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    // the row's own atom shares its molecule: with the
                    // same-molecule exclusion, one test drops both
                    if constexpr (kSameMol) keep[k] = live[k] & ~__ballot(pm[k] == moli);
                    else keep[k] = live[k] & __ballot(pu[k] != ui);
                }
                // the row's exclusions: each read once for all K candidates,
                // several reads in flight before the first compare
#pragma unroll 4
                for (int e = 0; e < ne; ++e) {
                    const int x = hex[e];
#pragma unroll
                    for (int k = 0; k < K; ++k) keep[k] &= __ballot(pu[k] != x);
                }
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    if (cb + kWave * k >= ncand) break;
                    // the distance test for every lane (no divergent branch
                    // around it), then the other conditions
                    bool in;
                    if constexpr (kKnown)
                        in = member_shifted(xi, yi, zi, px[k], py[k], pz[k], sx[k], sy[k], sz[k],
                                            rl2);
                    else
                        in = member(make_double4(xi, yi, zi, 0.0),
                                    make_double4(px[k], py[k], pz[k], 0.0), Lx, Ly, Lz, hx, hy,
                                    hz, rl2);
                    const uint64_t mask = keep[k] & __ballot(in);
                    if (__builtin_amdgcn_inverse_ballot_w64(mask)) {
                        // 32-bit slot index: the store takes the row's scalar
                        // base and one lane offset
                        const uint32_t p = (uint32_t)(hc + lanes_below(mask));
                        if (p < (uint32_t)cap) out[p] = (int)pe[k];
                    }
                    hc += __popcll(mask);
                }
                if (lane == h) mcnt = hc;
            } while (++h < h1);
            };
            if (known_shift) {
                if (same_mol) row_loop(BoolC<true>(), BoolC<true>());
                else row_loop(BoolC<true>(), BoolC<false>());
            } else {
                if (same_mol) row_loop(BoolC<false>(), BoolC<true>());
                else row_loop(BoolC<false>(), BoolC<false>());
            }
        }
        if (ncand == 0) range_of();
        // the slot table is rewritten for the next cell
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        h0 = h1;
    }
    if (lane < nh) {
        gbl(g.nrow)[myrow] = mcnt;
        const int stored = min(mcnt, cap);
        const int ty = mt | (gs_lo << kTypeBits);
        if (site) s_rec[myrow] = make_int4(mu, ty, stored, marow);
        else a_rec[myrow] = make_int4(mu, ty, stored, topo.hybrid[mt]);
    }
    // only a row that outgrew its capacity touches the status word (rare), so
    // thousands of waves do not serialise on one address
    if (lane < nh && mcnt > cap) atomicMax(&st->max_row[site ? 1 : 0], mcnt);
}

// One launch for both grids: waves [0, waves_a) build the atom list, the
// rest the site list; SA and SS are the stencil widths of the two grids.
template <int K, int SA, int SS>
__global__ __launch_bounds__(256) void k_lists_wave(const GridDev* __restrict__ grids,
                                                    int waves_a, int waves_total, int max_excl,
                                                    TopoDev topo,
                                                    const int* __restrict__ user2arow,
                                                    int4* __restrict__ a_rec,
                                                    int4* __restrict__ s_rec,
                                                    Status* __restrict__ st)
{
    __shared__ int slot_base[4][Stencil<(SA > SS ? SA : SS)>::kTab];
    __shared__ double slot_shift[4][3 * Stencil<(SA > SS ? SA : SS)>::kTab];
    __shared__ __align__(16) int slot_win[4][kWave * K];
    extern __shared__ int excl_lds[];
    // wave-uniform by construction; readfirstlane lets the compiler keep it
    // (and everything derived from it) in scalar registers
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int gw = blockIdx.x * 4 + wv;
    if (gw < waves_total) {                   // whole wave; no block barriers below
        const bool site = gw >= waves_a;
        const int lw = site ? gw - waves_a : gw;
        if (site)
            list_wave<K, SS>(grids[1], wv, lw, true, max_excl, topo, user2arow, a_rec, s_rec, st,
                             slot_base[wv], slot_shift[wv], slot_win[wv],
                             excl_lds);
        else
            list_wave<K, SA>(grids[0], wv, lw, false, max_excl, topo, user2arow, a_rec, s_rec,
                             st, slot_base[wv], slot_shift[wv], slot_win[wv],
                             excl_lds);
    }
    clear_bucket_counts(grids);   // last: the stores leave the start of the kernel alone
}

// Neighbour lists: one block per home cell (atom-grid cells first, then
// site-grid cells).  Rows are padded to the grid's capacity; the true count
// is stored even when it exceeds the capacity, so the host can regrow.
__global__ __launch_bounds__(kListBlock) void k_lists(const GridDev* __restrict__ grids,
                                                      int ncell_a, TopoDev topo,
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

    clear_bucket_counts(grids);
    const bool site = (int)blockIdx.x >= ncell_a;
    const GridDev& g = grids[site ? 1 : 0];
    const int c = site ? (int)blockIdx.x - ncell_a : (int)blockIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;

    if (threadIdx.x < 27) {
        // one lane per stencil slot: neighbour rank from the host-built table
        const int t = threadIdx.x;
        const int r = g.nbr[c * 27 + t];
        int cnt = -1, s0 = 0;
        if (r >= 0) {
            s0 = g.start[r];
            cnt = g.start[r + 1] - s0;
        }
        cell_start[t] = s0;
        cell_cnt[t] = cnt;
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
    const GeomDev& G = g.geom[g.cell_sys[c]];
    const double Lx = G.box[0], Ly = G.box[1], Lz = G.box[2];
    const double hx = G.half[0], hy = G.half[1], hz = G.half[2];
    const double rl2 = G.rl2;
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
                int eb = 0, ne = 0;
                if (topo.excl_off) {
                    eb = topo.excl_off[ui];
                    ne = min(topo.excl_off[ui + 1] - eb, kWave);
                }
                const int myex = lane < ne ? topo.excl_idx[eb + lane] : -1;
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
                        for (int k = 0; k < ne; ++k)
                            if (__shfl(myex, k) == uj) keep = false;
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
            const int tys = ty | (g.cell_sys[c] << kTypeBits);
            if (site) s_rec[row] = make_int4(u, tys, stored, user2arow[u]);
            else a_rec[row] = make_int4(u, tys, stored, topo.hybrid[ty]);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && blk_max > cap) atomicMax(&st->max_row[site ? 1 : 0], blk_max);
}

// Exact list statistics on demand: entries (sum of row lengths) and the
// longest row of each grid.  One block per grid.
__global__ __launch_bounds__(256) void k_list_stats(const GridDev* __restrict__ grids,
                                                    Status* __restrict__ st)
{
    __shared__ unsigned long long ssum[256 / kWave];
    __shared__ int smax[256 / kWave];
    const GridDev& g = grids[blockIdx.x];
    unsigned long long sum = 0ull;
    int mx = 0;
    RELRES_GLOBAL const int* gnrow = gbl(g.nrow);
    for (int r = threadIdx.x; r < g.members; r += blockDim.x) {
        const int c = gnrow[r];
        sum += (unsigned long long)c;
        mx = max(mx, c);
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        sum += __shfl_xor(sum, o);
        mx = max(mx, __shfl_xor(mx, o));
    }
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    if (lane == 0) {
        ssum[wave] = sum;
        smax[wave] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 256 / kWave; ++w) {
            ssum[0] += ssum[w];
            smax[0] = max(smax[0], smax[w]);
        }
        st->entries[blockIdx.x] = ssum[0];
        st->longest[blockIdx.x] = smax[0];
    }
}

// ---------------------------------------------------------------------------
// force kernel
// ---------------------------------------------------------------------------

// Coefficient table staged in LDS when it is small (ntypes <= kLdsTypes).
constexpr int kLdsTypes = 8;

template <typename S, bool EW>
struct CoefLds {
    PairCoef<S> c[kLdsTypes * kLdsTypes];
    PairCoef<double> c64[(EW && sizeof(S) != sizeof(double)) ? kLdsTypes * kLdsTypes : 1];
};

// Distances per type pair, staged when they are not uniform (PC).
template <typename S, bool PC>
struct CutLds {
    Cutoffs<S> c[PC ? kLdsTypes * kLdsTypes : 1];
    Cutoffs<double> c64[(PC && sizeof(S) != sizeof(double)) ? kLdsTypes * kLdsTypes : 1];
};

// The coefficient and distance rows of one row atom's type: pair-math
// coefficients, FP64 coefficients (energy and virial), and with per-pair
// distances (PC) the distance rows in both types.
template <typename S>
struct RowTab {
    const PairCoef<S>* c;
    const PairCoef<double>* c64;
    const Cutoffs<S>* cut;
    const Cutoffs<double>* cut64;
};

// A table of `count` T staged in LDS in two parts: stage_first reads word
// threadIdx.x (issued early, before the row record), stage_table writes it and
// copies any words beyond the first blockDim.x.
template <typename T>
__device__ __forceinline__ uint32_t stage_first(const T* __restrict__ src, int count)
{
    const int words = count * (int)(sizeof(T) / sizeof(uint32_t));
    return (int)threadIdx.x < words ? reinterpret_cast<const uint32_t*>(src)[threadIdx.x] : 0u;
}
template <typename T>
__device__ __forceinline__ void stage_table(T* dst, const T* __restrict__ src, int count,
                                            uint32_t first)
{
    const int words = count * (int)(sizeof(T) / sizeof(uint32_t));
    const uint32_t* s = reinterpret_cast<const uint32_t*>(src);
    uint32_t* d = reinterpret_cast<uint32_t*>(dst);
    if ((int)threadIdx.x < words) d[threadIdx.x] = first;
    for (int k = threadIdx.x + blockDim.x; k < words; k += blockDim.x) d[k] = s[k];
}

// Entries handled per lane per batch (see row_terms).
constexpr int kBatch = 2;
// ... and in forces-only launches of at least 8 entries per lane (issue-bound
// launches of large systems), where more gathers in flight per lane pay: the
// 256-replica batch's forces-only launch took 157 against 180 us, while every
// energy/virial launch and the launches of small systems were slower with 4.
constexpr int kBatchWide = 4;

constexpr uint32_t kNoEntry = 0xffffffffu;

// Periodic box of the system a row belongs to: edges and their reciprocals.
struct BoxV {
    double L[3], iL[3];
};

__device__ __forceinline__ BoxV row_box(const ForceArgs& a, int sys)
{
    BoxV b;
    if (a.nsys == 1) {
        for (int k = 0; k < 3; ++k) {
            b.L[k] = a.box[k];
            b.iL[k] = a.inv_box[k];
        }
    } else {
        for (int k = 0; k < 3; ++k) {
            b.L[k] = a.boxes[6 * sys + k];
            b.iL[k] = a.boxes[6 * sys + 3 + k];
        }
    }
    return b;
}

// Pair terms of one list entry, the FG part (CG = false, zero beyond r_s+) or
// the CG part (CG = true, zero beyond r_c+) of Eq. 20, with the neighbour's
// position already loaded.  Differences are taken in FP64 with the minimum
// image.  Force terms are evaluated in S and accumulated in TF; energy and
// virial terms are evaluated in FP64 and accumulated in FP64 (when they are
// requested, the FP32 force is rounded from the same FP64 terms).
template <bool CG, typename S, typename TF, bool EW, bool PC>
__device__ __forceinline__ void entry_terms(const BoxV& bx, const RowTab<S>& t,
                                            const Cutoffs<S>& cut_all,
                                            const Cutoffs<double>& cut64_all,
                                            double xi, double yi, double zi, uint32_t e,
                                            double px, double py, double pz,
                                            TF& fx, TF& fy, TF& fz, double* acc)
{
    if (e == kNoEntry) return;
    const int tj = (int)(e >> kIdxBits);
    const Cutoffs<double>& cut64 = PC ? t.cut64[tj] : cut64_all;
    const double rmax2 = CG ? cut64.rco2 : cut64.rso2;
    double dx = xi - px;
    double dy = yi - py;
    double dz = zi - pz;
    dx -= bx.L[0] * rint(dx * bx.iL[0]);
    dy -= bx.L[1] * rint(dy * bx.iL[1]);
    dz -= bx.L[2] * rint(dz * bx.iL[2]);
    const double r2d = dx * dx + dy * dy + dz * dz;
    if (!(r2d < rmax2)) return;
    if constexpr (sizeof(S) == sizeof(double) || EW) {
        // FP64 pair terms (full precision in FP64 mode; one Newton step when
        // they only feed energy/virial and FP32 forces)
        using M = MathF64<sizeof(S) == sizeof(double) ? 2 : 1>;
        double fpd, end;
        if constexpr (CG) cg_term<M>(t.c64[tj], cut64, r2d, fpd, end);
        else fg_term<M>(t.c64[tj], cut64, r2d, fpd, end);
        if constexpr (sizeof(TF) == sizeof(double)) {
            fx += fpd * dx;
            fy += fpd * dy;
            fz += fpd * dz;
        } else {
            const float fp = (float)fpd;
            fx += fp * (float)dx;
            fy += fp * (float)dy;
            fz += fp * (float)dz;
        }
        if constexpr (EW) {
            const double hf = 0.5 * fpd;
            acc[CG ? 1 : 0] += 0.5 * end;
            acc[2] += hf * dx * dx;
            acc[3] += hf * dy * dy;
            acc[4] += hf * dz * dz;
            acc[5] += hf * dx * dy;
            acc[6] += hf * dx * dz;
            acc[7] += hf * dy * dz;
        }
    } else {
        float fp, en;
        const Cutoffs<S>& cut = PC ? t.cut[tj] : cut_all;
        if constexpr (CG) cg_term<MathF32>(t.c[tj], cut, (float)r2d, fp, en);
        else fg_term<MathF32>(t.c[tj], cut, (float)r2d, fp, en);
        fx += fp * (float)dx;
        fy += fp * (float)dy;
        fz += fp * (float)dz;
    }
}

// Positions of a batch of entries (entry-less slots read atom 0, unused).
template <int B>
__device__ __forceinline__ void gather_batch(const ForceArgs& a, const uint32_t e[B],
                                             double px[B], double py[B], double pz[B])
{
#pragma unroll
    for (int u = 0; u < B; ++u) {
        const int uj = e[u] != kNoEntry ? (int)(e[u] & kIdxMask) : 0;
        px[u] = a.pos[3 * uj];
        py[u] = a.pos[3 * uj + 1];
        pz[u] = a.pos[3 * uj + 2];
    }
}

// Entries start, start + G, ... below cnt of one list row, B per lane at
// a time: their list loads, then their position gathers, are issued together
// before any pair term is computed.
template <bool CG, typename S, typename TF, bool EW, bool PC, int B>
__device__ __forceinline__ void row_terms(const ForceArgs& a, const BoxV& bx,
                                          const RowTab<S>& t,
                                          const Cutoffs<S>& cut, const Cutoffs<double>& cut64,
                                          double xi, double yi, double zi,
                                          const int* __restrict__ lst, int start, int cnt, int G,
                                          TF& fx, TF& fy, TF& fz, double* acc)
{
    for (int base = start; base < cnt; base += G * B) {
        uint32_t e[B];
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int k = base + u * G;
            e[u] = k < cnt ? (uint32_t)lst[k] : kNoEntry;
        }
        double px[B], py[B], pz[B];
        gather_batch<B>(a, e, px, py, pz);
#pragma unroll
        for (int u = 0; u < B; ++u)
            entry_terms<CG, S, TF, EW, PC>(bx, t, cut, cut64, xi, yi, zi, e[u], px[u], py[u],
                                           pz[u], fx, fy, fz, acc);
    }
}


// ---------------------------------------------------------------------------
// Energy/virial reduction across the blocks of one force launch
// ---------------------------------------------------------------------------
// Each block's 8 partial sums (energy FG, CG, virial xx yy zz xy xz yz) are
// published as one record of 16 64-bit words: the high and low 32-bit halves
// of every double, each paired with a 32-bit launch tag.  64-bit stores are
// single-copy atomic, so a reader that sees the current tag in a word sees
// that word's payload; no store ever has to be waited for, and no atomic
// read-modify-write (which serialise on one address) is needed.  The tag is
// the device epoch + 1; the epoch advances once per launch.
//
// Blocks b with b % 16 == g form group g (16 groups: fewer records for each
// group's waiting block to poll than with 8, and still one poll round for the
// 16 group records).  The highest-numbered block of each group waits for the
// records of the rest of its group and publishes the group sum; block nb-1
// (the highest of all) then waits for the group records and writes energy
// and virial.  A waiting block only ever waits for blocks with
// lower numbers, which the hardware dispatched before it, so every wait ends;
// it is bounded anyway (a.spin_limit polls; a negative limit gives up at
// once), after which energy and virial are set to NaN and the status counts
// the failure, which the host reports (relres_sync, relres_check_lists).
// Sums are taken in a fixed order: the result does not depend on which block
// finished when.
constexpr int kRecWords = 16;

// Writes one record: called by the whole block, `v` valid in threads 0..7
// (component threadIdx.x).  Lanes 0..15 of wave 0 store word threadIdx.x, so
// the record goes out as one contiguous 128-byte write, written through to
// the level all XCDs share.
__device__ __forceinline__ void put_record(unsigned long long* rec, double v, unsigned tag)
{
    if (threadIdx.x < 64) {
        const double c = __shfl(v, (int)(threadIdx.x >> 1));
        const unsigned long long bits = (unsigned long long)__double_as_longlong(c);
        const unsigned long long half = (threadIdx.x & 1) ? (bits & 0xffffffffull) : (bits >> 32);
        const unsigned long long word = ((unsigned long long)tag << 32) | half;
        if (threadIdx.x < kRecWords)
            __hip_atomic_store(rec + threadIdx.x, word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Waits for `count` records (record m at rec + (first + stride*m) * 16 words)
// to carry `tag` and adds them up.  Sixteen consecutive lanes read the sixteen
// words of one record, so every load instruction covers whole records.  On
// return, even lanes hold their record-word pair's component (t % 16) / 2
// summed over their records in v[]; odd lanes hold zeros.  Sets *failed if a
// wait gave up.
template <int kPollBatch>      // records polled per thread at once
__device__ __forceinline__ void gather_records(const unsigned long long* rec, int first, int stride,
                                               int count, unsigned tag, int spin_limit,
                                               double v[8], int* failed)
{
    const int t = (int)threadIdx.x;
    const int word = t & (kRecWords - 1);
    const int comp = word >> 1;
    double sum = 0.0;
    for (int base = 0; base < count; base += (kForceBlock / kRecWords) * kPollBatch) {
        // every slot loads on every poll (slots past `count` re-read the
        // first record), so all loads of a poll are in flight together; a
        // record already complete is final for this launch
        size_t off[kPollBatch];
        bool valid[kPollBatch];
#pragma unroll
        for (int u = 0; u < kPollBatch; ++u) {
            const int m = base + t / kRecWords + (kForceBlock / kRecWords) * u;
            valid[u] = m < count;
            off[u] = (size_t)(first + stride * (valid[u] ? m : 0)) * kRecWords + word;
        }
        unsigned long long w[kPollBatch];
        for (int it = 0;; ++it) {
#pragma unroll
            for (int u = 0; u < kPollBatch; ++u)
                w[u] = __hip_atomic_load(rec + off[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            bool pending = false;
#pragma unroll
            for (int u = 0; u < kPollBatch; ++u)
                pending |= valid[u] && (unsigned)(w[u] >> 32) != tag;
            pending |= spin_limit < 0 && count > 0;   // give up at once
            if (!pending) break;
            if (it >= spin_limit) {
                *failed = 1;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
#pragma unroll
        for (int u = 0; u < kPollBatch; ++u) {
            const unsigned lo = (unsigned)__shfl_down((unsigned)(w[u] & 0xffffffffull), 1);
            if (!(word & 1) && valid[u])
                sum += __longlong_as_double((long long)(((w[u] & 0xffffffffull) << 32) | lo));
        }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = (!(word & 1) && k == comp) ? sum : 0.0;
}

// Fixed-order block reduction of v[8]: result in threads 0..7 (component
// threadIdx.x) as the return value; `extra` (threads 0..7) is added last.
__device__ __forceinline__ double block_reduce8(const double v[8], double extra,
                                                double (*red)[kForceBlock / 64])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double s = wave_sum8(v);
    if (lane < 8) red[wave_sum8_lane(lane)][wave] = s;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x < 8) {
        for (int w = 0; w < kForceBlock / 64; ++w) t += red[threadIdx.x][w];
        t += extra;
    }
    __syncthreads();
    return t;
}

__device__ void ew_finish(const ForceArgs& a, const double acc[8], unsigned tag)
{
    __shared__ double red[8][kForceBlock / 64];
    __shared__ int failed;
    const int nb = (int)gridDim.x;
    const int b = (int)blockIdx.x;
    const int g = b % kEwGroups;
    const int ngroups = nb < kEwGroups ? nb : kEwGroups;
    const int last_in_group = g + kEwGroups * ((nb - 1 - g) / kEwGroups);

    if (threadIdx.x == 0) failed = 0;
    const double mine = block_reduce8(acc, 0.0, red);
    // records: blocks [0, nb), groups [nb, nb + 8)
    unsigned long long* grec = a.ew_rec + (size_t)nb * kRecWords;
    if (b != last_in_group) {
        put_record(a.ew_rec + (size_t)b * kRecWords, mine, tag);
        return;
    }
    // group g: members g, g+8, ..., b-8 (in that order), then this block
    double v[8];
    // records per thread per poll: as few loads as cover the group in one
    // round (a poll's loads queue on this one CU's memory pipeline, so extra
    // slots that re-read a record cost time: 16 per thread took 0.5 us more
    // than 8 for 71 records)
    const int count = b / kEwGroups;
    constexpr int kSlots = kForceBlock / kRecWords;      // records per load instruction
    if (count <= 2 * kSlots)
        gather_records<2>(a.ew_rec, g, kEwGroups, count, tag, a.spin_limit, v, &failed);
    else if (count <= 4 * kSlots)
        gather_records<4>(a.ew_rec, g, kEwGroups, count, tag, a.spin_limit, v, &failed);
    else if (count <= 8 * kSlots)
        gather_records<8>(a.ew_rec, g, kEwGroups, count, tag, a.spin_limit, v, &failed);
    else
        gather_records<16>(a.ew_rec, g, kEwGroups, count, tag, a.spin_limit, v, &failed);
    const double gsum = block_reduce8(v, mine, red);
    if (b != nb - 1) {
        put_record(grec + (size_t)g * kRecWords, failed ? __builtin_nan("") : gsum, tag);
        if (threadIdx.x == 0 && failed) atomicAdd(a.ew_failed, 1u);
        return;
    }
    // final block: the group sums in group order.  The other groups' records
    // are gathered (groups 0..ngroups-1 except g, which is this block's own);
    // to keep the order fixed, the own group's sum is slotted in at its place.
    __shared__ double gred[kEwGroups][8];
    if (threadIdx.x < 8) gred[g][threadIdx.x] = gsum;
    {
        const int t = (int)threadIdx.x;
        const int q = t / kRecWords, word = t & (kRecWords - 1);
        unsigned long long w = 0;
        if (q < ngroups && q != g) {
            for (int it = 0;; ++it) {
                w = __hip_atomic_load(grec + (size_t)q * kRecWords + word, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
                if ((unsigned)(w >> 32) == tag && a.spin_limit >= 0) break;
                if (it >= a.spin_limit) {
                    failed = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        const unsigned lo = (unsigned)__shfl_down((unsigned)(w & 0xffffffffull), 1);
        if (q < ngroups && q != g && !(word & 1))
            gred[q][word >> 1] = __longlong_as_double((long long)(((w & 0xffffffffull) << 32) | lo));
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        double t = 0.0;
        for (int q = 0; q < ngroups; ++q) t += gred[q][threadIdx.x];
        red[threadIdx.x][0] = t;
    }
    __syncthreads();
    const bool bad = failed != 0;
    if (threadIdx.x == 0 && bad) atomicAdd(a.ew_failed, 1u);
    if (threadIdx.x < 8) {
        const double val = bad ? __builtin_nan("") : red[threadIdx.x][0];
        if (threadIdx.x < 2 && a.energy) a.energy[1 + threadIdx.x] = val;
        if (threadIdx.x >= 2 && a.virial) a.virial[threadIdx.x - 2] = val;
    }
    if (threadIdx.x == 0) {
        if (a.energy) a.energy[0] = bad ? __builtin_nan("") : red[0][0] + red[1][0];
        __hip_atomic_store(a.epoch, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

template <typename S, typename TF, bool EW, bool LDS, bool PC, int B>
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

    // the first words of the LDS tables are read before the row record, so
    // the two reads overlap (written to LDS once the record is in)
    const PairCoef<S>* coef_g = (const PairCoef<S>*)(sizeof(S) == 8 ? a.coef64 : a.coef32);
    const Cutoffs<S>* pcut_g = (const Cutoffs<S>*)(sizeof(S) == 8 ? (const void*)a.pcut64
                                                                   : (const void*)a.pcut32);
    const int np = a.ntypes * a.ntypes;
    uint32_t stg[4] = {0u, 0u, 0u, 0u};
    if constexpr (LDS) {
        stg[0] = stage_first(coef_g, np);
        if constexpr (EW && sizeof(S) != sizeof(double))
            stg[1] = stage_first((const PairCoef<double>*)a.coef64, np);
        if constexpr (PC) {
            stg[2] = stage_first(pcut_g, np);
            if constexpr (sizeof(S) != sizeof(double)) stg[3] = stage_first(a.pcut64, np);
        }
    }

    unsigned tag = 0;
    if constexpr (EW) {
        // tag 0 is never used: it marks a cleared record.  The epoch is an
        // ordinary load: only the previous launch wrote it (this launch writes
        // it after every block has published, i.e. after every block read
        // it), and the kernel boundary makes that write visible.  A
        // device-coherent atomic load from every wave cost 0.2 us per launch.
        tag = a.epoch[0] + 1u;
        tag += tag == 0u;
    }
    // The row's own list (the atom list for rows of ordinary atoms, the site
    // list for rows of hybrid atoms) does not depend on the row record, so its
    // first entries are loaded together with the record.  Slots past the row's
    // count read the row's padding (in bounds) and are dropped once the count
    // is known.
    const bool live = rb ? row < a.n_srow : row < a.n_arow;
    const int* own_list = rb ? a.s_list + (size_t)row * a.s_cap : a.a_list + (size_t)row * a.a_cap;
    const int own_cap = rb ? a.s_cap : a.a_cap;
    uint32_t e_own[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
        const int k = sub + u * G;
        e_own[u] = (live && k < own_cap) ? (uint32_t)own_list[k] : kNoEntry;
    }
    int4 rec = make_int4(-1, 0, 0, 1);
    if (live) rec = rb ? a.s_rec[row] : a.a_rec[row];
    // FG entries: for a hybrid row they sit in the atom-list row named by the
    // record (loaded together with that row's count)
    uint32_t e_fg[B];
    int cnt_a = rec.z;
    if (rb) {
#pragma unroll
        for (int u = 0; u < B; ++u) e_fg[u] = kNoEntry;
        cnt_a = 0;
        if (live) {
            const int* fl = a.a_list + (size_t)rec.w * a.a_cap;
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int k = sub + u * G;
                if (k < a.a_cap) e_fg[u] = (uint32_t)fl[k];
            }
            cnt_a = a.a_rec[rec.w].z;
        }
    } else {
#pragma unroll
        for (int u = 0; u < B; ++u) e_fg[u] = e_own[u];
    }

    const PairCoef<S>* coef;
    const PairCoef<double>* coef64;
    const Cutoffs<S>* pcut = nullptr;
    const Cutoffs<double>* pcut64 = nullptr;
    if constexpr (LDS) {
        __shared__ CoefLds<S, EW> tab;
        __shared__ CutLds<S, PC> ctab;
        stage_table(tab.c, coef_g, np, stg[0]);
        if constexpr (EW && sizeof(S) != sizeof(double))
            stage_table(tab.c64, (const PairCoef<double>*)a.coef64, np, stg[1]);
        if constexpr (PC) {
            stage_table(ctab.c, pcut_g, np, stg[2]);
            if constexpr (sizeof(S) != sizeof(double)) stage_table(ctab.c64, a.pcut64, np, stg[3]);
        }
        __syncthreads();
        coef = tab.c;
        if constexpr (EW && sizeof(S) != sizeof(double)) coef64 = tab.c64;
        else coef64 = (const PairCoef<double>*)tab.c;
        if constexpr (PC) {
            pcut = ctab.c;
            if constexpr (sizeof(S) != sizeof(double)) pcut64 = ctab.c64;
            else pcut64 = (const Cutoffs<double>*)ctab.c;
        }
    } else {
        coef = coef_g;
        coef64 = (const PairCoef<double>*)a.coef64;
        if constexpr (PC) {
            pcut = pcut_g;
            pcut64 = a.pcut64;
        }
    }

    TF fx = TF(0), fy = TF(0), fz = TF(0);
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const bool own = rb ? rec.x >= 0 : (rec.x >= 0 && rec.w == 0);   // hybrid atom rows belong to the site range
    if (own) {
        const int ui = rec.x, ti = rec.y & ((1 << kTypeBits) - 1);
        const int cnt_s = rb ? rec.z : 0;
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int k = sub + u * G;
            if (k >= cnt_a) e_fg[u] = kNoEntry;
            if (k >= cnt_s) e_own[u] = kNoEntry;
        }
        const double xi = a.pos[3 * ui], yi = a.pos[3 * ui + 1], zi = a.pos[3 * ui + 2];
        // the first batches of both parts: all gathers before any arithmetic
        double fxp[B], fyp[B], fzp[B], sxp[B], syp[B], szp[B];
        gather_batch<B>(a, e_fg, fxp, fyp, fzp);
        if (rb) gather_batch<B>(a, e_own, sxp, syp, szp);
        // the row's box (several systems: a read) after the gathers, so the
        // wave does not wait for it before issuing them
        const BoxV bx = row_box(a, rec.y >> kTypeBits);
        const int ro = ti * a.ntypes;
        const RowTab<S> rt{coef + ro, coef64 + ro, PC ? pcut + ro : nullptr,
                           PC ? pcut64 + ro : nullptr};
#pragma unroll
        for (int u = 0; u < B; ++u)
            entry_terms<false, S, TF, EW, PC>(bx, rt, cut, cut64, xi, yi, zi, e_fg[u], fxp[u],
                                              fyp[u], fzp[u], fx, fy, fz, acc);
        if (rb) {
#pragma unroll
            for (int u = 0; u < B; ++u)
                entry_terms<true, S, TF, EW, PC>(bx, rt, cut, cut64, xi, yi, zi, e_own[u],
                                                 sxp[u], syp[u], szp[u], fx, fy, fz, acc);
        }
        // the rest of both rows
        const int ar = rb ? rec.w : row;
        const int rest = sub + B * G;
        row_terms<false, S, TF, EW, PC, B>(a, bx, rt, cut, cut64, xi, yi, zi,
                                        a.a_list + (size_t)ar * a.a_cap, rest, cnt_a, G, fx, fy,
                                        fz, acc);
        if (rb)
            row_terms<true, S, TF, EW, PC, B>(a, bx, rt, cut, cut64, xi, yi, zi,
                                           a.s_list + (size_t)row * a.s_cap, rest, cnt_s, G, fx,
                                           fy, fz, acc);
    }
    fx = group_sum(fx, G);
    fy = group_sum(fy, G);
    fz = group_sum(fz, G);
    if (own && sub == 0) {
        TF* F = (TF*)a.forces;
        F[3 * rec.x] = fx;
        F[3 * rec.x + 1] = fy;
        F[3 * rec.x + 2] = fz;
    }
    if constexpr (EW) {
        if (a.nsys == 1) {
            ew_finish(a, acc, tag);
        } else {
            // several systems (rows are grouped by system): a wave whose own
            // rows all belong to one system adds its lanes and writes one
            // record; a wave across a system boundary (rare) writes every
            // row's partials.  A second kernel adds each system's records.
            const int lane = (int)threadIdx.x & (kWave - 1);
            const size_t wrec = (rb ? (size_t)a.blocks_a * (kForceBlock / kWave) : 0) +
                                (size_t)logical * (kForceBlock / kWave) + (threadIdx.x / kWave);
            const int sys_row = own ? (rec.y >> kTypeBits) : -1;
            const uint64_t own_mask = __ballot(own);
            if (own_mask == 0ull) {
                if (lane == 0) a.wave_sys[wrec] = -2;
            } else {
                const int s0 = __builtin_amdgcn_readlane(sys_row, __ffsll((long long)own_mask) - 1);
                if (__ballot(own && sys_row != s0) == 0ull) {
                    const double ws = wave_sum8(acc);
                    if (lane < 8) a.wave_ew[8 * wrec + wave_sum8_lane(lane)] = ws;
                    if (lane == 0) a.wave_sys[wrec] = s0;
                } else {
#pragma unroll
                    for (int k = 0; k < 8; ++k) acc[k] = group_sum(acc[k], G);
                    if (live && sub == 0) {
                        double* out = a.row_ew + 8 * (size_t)(rb ? a.n_arow + row : row);
#pragma unroll
                        for (int k = 0; k < 8; ++k) out[k] = own ? acc[k] : 0.0;
                    }
                    if (lane == 0) a.wave_sys[wrec] = -1;
                }
            }
        }
    }
}


__global__ void k_zero_outputs(double* energy, double* virial, int nsys)
{
    for (int t = threadIdx.x; t < 6 * nsys; t += blockDim.x) {
        if (energy && t < 3 * nsys) energy[t] = 0.0;
        if (virial) virial[t] = 0.0;
    }
}

// Energy and virial of every system (one block per system) from the per-row
// partials of the force kernel: the system's atom-list rows, then its
// site-list rows, each thread in row order, then a fixed-order block sum.
// One block per system: the records of the waves that hold its rows (wave
// w of a kind holds rows w * rpw .. w * rpw + rpw - 1 of that kind, rpw =
// 64 / lanes per row), and for a wave across a system boundary the partials
// of its rows in this system; fixed order, so results are deterministic.
constexpr int kSysLoads = 4;

__global__ __launch_bounds__(256) void k_reduce_sys_ew(const GridDev* __restrict__ grids,
                                                       int ngrids, ForceArgs a,
                                                       double* __restrict__ energy,
                                                       double* __restrict__ virial)
{
    __shared__ double red[8][4];
    const int sy = (int)blockIdx.x;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    // the system's waves of both kinds (atom rows, then site rows) as one
    // range: both kinds' row ranges are read first, then kSysLoads waves per
    // thread per round have their system tags and records requested before
    // any is used (a record is read whatever its tag says); the waves whose
    // rows are all this system's (tag sy) are added here
    // (the grid array always has two entries, so both kinds' ranges are read
    // unconditionally, as scalar loads all in flight together)
    int w0[2] = {0, 0}, nw[2] = {0, 0}, rpw[2] = {1, 1}, r0[2] = {0, 0}, r1[2] = {0, 0};
    {
        RELRES_GLOBAL const GridDev* gg = gbl(grids);
        RELRES_GLOBAL const GeomDev* ge0 = gbl(gg[0].geom);
        RELRES_GLOBAL const GeomDev* ge1 = gbl(gg[1].geom);
        const int base[2] = {ge0[sy].row_base, ge1[sy].row_base};
        const int mem[2] = {ge0[sy].members, ngrids > 1 ? ge1[sy].members : 0};
#pragma unroll
        for (int kind = 0; kind < 2; ++kind) {
            rpw[kind] = kWave >> (kind ? a.log_lanes_b : a.log_lanes_a);
            r0[kind] = base[kind];
            r1[kind] = base[kind] + mem[kind];
            w0[kind] = r0[kind] / rpw[kind];
            nw[kind] = mem[kind] > 0 ? (r1[kind] - 1) / rpw[kind] - w0[kind] + 1 : 0;
        }
    }
    const size_t woff1 = (size_t)a.blocks_a * (kForceBlock / kWave);
    const int total = nw[0] + nw[1];
    for (int jb = (int)threadIdx.x; jb < total; jb += 256 * kSysLoads) {
        int ws[kSysLoads];
        double4 q[kSysLoads][2];
#pragma unroll
        for (int u = 0; u < kSysLoads; ++u) {
            const int j = min(jb + 256 * u, total - 1);
            const size_t wg = j < nw[0] ? (size_t)(w0[0] + j) : woff1 + (size_t)(w0[1] + j - nw[0]);
            const double4* p = reinterpret_cast<const double4*>(a.wave_ew + 8 * wg);
            ws[u] = jb + 256 * u < total ? a.wave_sys[wg] : -2;
            q[u][0] = p[0];
            q[u][1] = p[1];
        }
#pragma unroll
        for (int u = 0; u < kSysLoads; ++u) {
            if (ws[u] == sy) {
                v[0] += q[u][0].x; v[1] += q[u][0].y; v[2] += q[u][0].z; v[3] += q[u][0].w;
                v[4] += q[u][1].x; v[5] += q[u][1].y; v[6] += q[u][1].z; v[7] += q[u][1].w;
            }
        }
    }
    // A wave across a system boundary (tag -1) left partials per row; only
    // the first or the last wave of a kind's range can be one.  Their rows of
    // this system, one row per thread, all four waves' loads issued together.
    {
        int wsb[4];
        bool use[4];
        double4 qb[4][2];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int kind = q >> 1, e = q & 1;
            const bool any = nw[kind] > 0 && (e == 0 || nw[kind] > 1);
            const int w = e == 0 ? w0[kind] : w0[kind] + nw[kind] - 1;
            const int lo = max(w * rpw[kind], r0[kind]), hi = min((w + 1) * rpw[kind], r1[kind]);
            const int r = lo + (int)threadIdx.x;
            use[q] = any && r < hi;
            wsb[q] = any ? a.wave_sys[(kind ? woff1 : 0) + (size_t)w] : -2;
            const size_t ri = any ? (kind ? (size_t)a.n_arow : 0) + (size_t)(use[q] ? r : lo) : 0;
            const double4* p = reinterpret_cast<const double4*>(a.row_ew + 8 * ri);
            qb[q][0] = p[0];
            qb[q][1] = p[1];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (use[q] && wsb[q] == -1) {
                v[0] += qb[q][0].x; v[1] += qb[q][0].y; v[2] += qb[q][0].z; v[3] += qb[q][0].w;
                v[4] += qb[q][1].x; v[5] += qb[q][1].y; v[6] += qb[q][1].z; v[7] += qb[q][1].w;
            }
        }
    }
    {
        const double s = wave_sum8(v);
        const int lane = (int)threadIdx.x & 63;
        if (lane < 8) red[wave_sum8_lane(lane)][threadIdx.x >> 6] = s;
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        const int k = threadIdx.x;
        const double t = red[k][0] + red[k][1] + red[k][2] + red[k][3];
        if (k < 2 && energy) energy[3 * sy + 1 + k] = t;
        if (k >= 2 && virial) virial[6 * sy + k - 2] = t;
        red[k][0] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0 && energy) energy[3 * sy] = red[0][0] + red[1][0];
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

hipError_t launch_bin(int n, const double* pos, TopoDev topo, GridDev* grids_dev, double4* wpos,
                      int2* key_a, int2* key_s, Status* st, bool check_moved, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bin, dim3((n + 255) / 256), dim3(256), 0, s, n, pos, topo, grids_dev,
                       wpos, key_a, key_s, st, check_moved ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_moved(int n, const double* pos, TopoDev topo, const GridDev* grids_dev,
                        const double4* wpos, Status* st, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_moved, dim3((n + 255) / 256), dim3(256), 0, s, n, pos, topo, grids_dev,
                       wpos, st);
    return hipGetLastError();
}

int scan_segments(int ncell) { return (ncell + kScanSeg - 1) / kScanSeg; }

hipError_t launch_scan(GridDev* grids_dev, int ngrids, int ncell_a, int ncell_s, int* seg_tot,
                       hipStream_t s)
{
    const int nseg0 = scan_segments(ncell_a), nseg1 = ngrids > 1 ? scan_segments(ncell_s) : 0;
    if (nseg0 <= 1 && nseg1 <= 1) {
        hipLaunchKernelGGL(k_scan, dim3(ngrids), dim3(kScanThreads), 0, s, grids_dev);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_totals, dim3(nseg0 + nseg1), dim3(kScanThreads), 0, s, grids_dev,
                       nseg0, seg_tot);
    hipLaunchKernelGGL(k_scan_segments, dim3(nseg0 + nseg1), dim3(kScanThreads), 0, s, grids_dev,
                       nseg0, seg_tot);
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

hipError_t launch_cellsort(GridDev* grids_dev, int ncell_a, int ncell_total, long long members,
                           const double4* wpos, TopoDev topo, int* user2arow, hipStream_t s)
{
    // a few members per cell (mean below 8): 4 cells per wave
    const bool small = (long long)members < 8LL * ncell_total;
    const int waves_per_block = 4;
    const int cells_per_block = waves_per_block * (small ? 4 : 1);
    int blocks = (ncell_total + cells_per_block - 1) / cells_per_block;
    if (blocks > 65535) blocks = 65535;
    if (blocks < 1) blocks = 1;
    if (small)
        hipLaunchKernelGGL(k_cellsort<16>, dim3(blocks), dim3(64 * waves_per_block), 0, s,
                           grids_dev, ncell_a, ncell_total, wpos, topo, user2arow);
    else
        hipLaunchKernelGGL(k_cellsort<64>, dim3(blocks), dim3(64 * waves_per_block), 0, s,
                           grids_dev, ncell_a, ncell_total, wpos, topo, user2arow);
    return hipGetLastError();
}

hipError_t launch_place(GridDev* grids_dev, int ncell_a, int ncell_s, long long members, int n,
                        const int2* key_a, const int2* key_s, const double4* wpos, TopoDev topo,
                        int* user2arow, hipStream_t s)
{
    // a few members per cell (mean below 8): 4 cells per wave, as k_cellsort
    const bool small = members < 8LL * (ncell_a + ncell_s);
    const int cells = (kPlaceThreads / kWave) * (small ? 4 : 1);
    const int blocks_a = (ncell_a + cells - 1) / cells, blocks_s = (ncell_s + cells - 1) / cells;
    if (blocks_a + blocks_s == 0) return hipSuccess;
    if (small)
        hipLaunchKernelGGL(k_place<16>, dim3(blocks_a + blocks_s), dim3(kPlaceThreads), 0, s,
                           grids_dev, blocks_a, n, key_a, key_s, wpos, topo, user2arow);
    else
        hipLaunchKernelGGL(k_place<64>, dim3(blocks_a + blocks_s), dim3(kPlaceThreads), 0, s,
                           grids_dev, blocks_a, n, key_a, key_s, wpos, topo, user2arow);
    return hipGetLastError();
}

int list_candidates(int total_waves, int cand)
{
    if (cand == 2 || cand == 4) return cand;
    // RELRES_LIST_CANDIDATES=2|4 overrides the automatic choice (tuning runs)
    if (const char* e = std::getenv("RELRES_LIST_CANDIDATES")) {
        if (e[0] == '2' && e[1] == 0) return 2;
        if (e[0] == '4' && e[1] == 0) return 4;
    }
    // all waves resident at once (about 3 per SIMD): more candidates per lane
    return total_waves <= kResidentListWaves ? 4 : 2;
}

hipError_t launch_lists(GridDev* grids_dev, int ncell_a, int ncell_s, int waves_a, int waves_s,
                        TopoDev topo, const int* user2arow, int4* a_rec, int4* s_rec, Status* st,
                        bool per_wave, int cand, int stencil_a, int stencil_s, hipStream_t s)
{
    if (per_wave || stencil_a != 3 || stencil_s != 3) {
        const int total = waves_a + waves_s;
        if (total == 0) return hipSuccess;
        const int mx = topo.excl_off ? topo.max_excl : 0;
        const size_t dyn = sizeof(int) * 4 * kRowsPerWave * (size_t)mx;
        const bool k4 = list_candidates(total, cand) == 4;
        const dim3 grid((total + 3) / 4), block(256);
#define RELRES_LISTS(K, SA, SS)                                                                   \
        hipLaunchKernelGGL((k_lists_wave<K, SA, SS>), grid, block, dyn, s, grids_dev, waves_a, \
                           total, mx, topo, user2arow, a_rec, s_rec, st)
        const int sel = (k4 ? 4 : 0) | (stencil_a == 5 ? 2 : 0) | (stencil_s == 5 ? 1 : 0);
        switch (sel) {
        case 0: RELRES_LISTS(2, 3, 3); break;
        case 1: RELRES_LISTS(2, 3, 5); break;
        case 2: RELRES_LISTS(2, 5, 3); break;
        case 3: RELRES_LISTS(2, 5, 5); break;
        case 4: RELRES_LISTS(4, 3, 3); break;
        case 5: RELRES_LISTS(4, 3, 5); break;
        case 6: RELRES_LISTS(4, 5, 3); break;
        default: RELRES_LISTS(4, 5, 5); break;
        }
#undef RELRES_LISTS
        return hipGetLastError();
    }
    if (ncell_a + ncell_s == 0) return hipSuccess;
    hipLaunchKernelGGL(k_lists, dim3(ncell_a + ncell_s), dim3(kListBlock), 0, s, grids_dev,
                       ncell_a, topo, user2arow, a_rec, s_rec, st);
    return hipGetLastError();
}

// One force launch; forces-only launches of wide rows take kBatchWide entries
// per lane per batch.
template <typename S, typename TF, bool EW, bool LDS, bool PC>
void launch_force_kernel(const ForceArgs& a, const double* cut64, dim3 grid, dim3 block,
                         hipStream_t s)
{
    if constexpr (!EW) {
        if (a.wide_batch) {
            hipLaunchKernelGGL((k_forces<S, TF, EW, LDS, PC, kBatchWide>), grid, block, 0, s, a,
                               cut_as<S>(cut64), cut_as<double>(cut64));
            return;
        }
    }
    hipLaunchKernelGGL((k_forces<S, TF, EW, LDS, PC, kBatch>), grid, block, 0, s, a,
                       cut_as<S>(cut64), cut_as<double>(cut64));
}

hipError_t launch_forces(const ForceArgs& a, const double* cut64, bool per_pair, int pair_math,
                         int precision, bool ew, hipStream_t s)
{
    const dim3 grid(a.blocks_a + a.blocks_b), block(kForceBlock);
    const bool lds = a.ntypes <= kLdsTypes;
#define RELRES_LAUNCH_PC(S, TF, EW, PC)                                                          \
    do {                                                                                         \
        if (lds)                                                                                 \
            launch_force_kernel<S, TF, EW, true, PC>(a, cut64, grid, block, s);                  \
        else                                                                                     \
            launch_force_kernel<S, TF, EW, false, PC>(a, cut64, grid, block, s);                 \
    } while (0)
#define RELRES_LAUNCH(S, TF, EW)                                                                 \
    do {                                                                                         \
        if (per_pair) RELRES_LAUNCH_PC(S, TF, EW, true);                                         \
        else RELRES_LAUNCH_PC(S, TF, EW, false);                                                 \
    } while (0)
    if (precision == 64) {
        if (ew) RELRES_LAUNCH(double, double, true); else RELRES_LAUNCH(double, double, false);
    } else if (pair_math == 64) {
        if (ew) RELRES_LAUNCH(double, float, true); else RELRES_LAUNCH(double, float, false);
    } else {
        if (ew) RELRES_LAUNCH(float, float, true); else RELRES_LAUNCH(float, float, false);
    }
#undef RELRES_LAUNCH
#undef RELRES_LAUNCH_PC
    return hipGetLastError();
}

hipError_t launch_list_stats(GridDev* grids_dev, int ngrids, Status* st, hipStream_t s)
{
    hipLaunchKernelGGL(k_list_stats, dim3(ngrids), dim3(256), 0, s, grids_dev, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// backward (adjoint) pass
// ---------------------------------------------------------------------------
// J = e_bar E + sum_i g_i . F_i.  Per ordered pair (i, j) of a list row, with
// d = x_i - x_j, fpair = -u~'(r)/r (F_i gets fpair d) and
// hc = (d fpair/dr)/r:
//   dJ/dx_i += -e_bar fpair d + fpair (g_i - g_j) + hc ((g_i - g_j) . d) d
//   dJ/dP_{t_i t_j} += e_bar u~_P / 2 + (g_i . d) fpair_P
// where u~_P, fpair_P are the pair terms evaluated with the derivative record
// of parameter P (the terms are linear in the record's coefficients).  Each
// unordered pair appears in both rows, hence the half energy weight.

// FG part with the Hessian factor, FP64.
__device__ __forceinline__ void fg_terms2(const PairCoef<double>& c, const Cutoffs<double>& cut,
                                          double r2, double& fpair, double& en, double& hc)
{
    using M = MathF64<2>;
    if (r2 < cut.rsi2) {
        const double r2i = M::recip(r2);
        const double r6i = r2i * r2i * r2i;
        fpair = r6i * (c.fg_c12 * r6i - c.fg_c6) * r2i;
        en = r6i * (c.fg_e12 * r6i - c.fg_e6) - c.fg_shift;
        hc = r2i * r2i * r6i * (8.0 * c.fg_c6 - 14.0 * c.fg_c12 * r6i);
    } else {
        double r, ir;
        M::root(r2, r, ir);
        const double d = r - cut.rsi;
        const double dp = c.fg_g[1] + d * (2.0 * c.fg_g[2] + d * (3.0 * c.fg_g[3] + d * (4.0 * c.fg_g[4])));
        const double dpp = 2.0 * c.fg_g[2] + d * (6.0 * c.fg_g[3] + d * (12.0 * c.fg_g[4]));
        fpair = -dp * ir;
        en = c.fg_g[0] + d * (c.fg_g[1] + d * (c.fg_g[2] + d * (c.fg_g[3] + d * c.fg_g[4]))) - c.fg_shift;
        hc = (-dpp - fpair) * ir * ir;
    }
}

// CG part with the Hessian factor, FP64.
__device__ __forceinline__ void cg_terms2(const PairCoef<double>& c, const Cutoffs<double>& cut,
                                          double r2, double& fpair, double& en, double& hc)
{
    using M = MathF64<2>;
    if (r2 < cut.rsi2) {
        fpair = 0.0;
        en = c.sp_g0 - c.sp_shift;
        hc = 0.0;
    } else if (r2 < cut.rso2) {
        double r, ir;
        M::root(r2, r, ir);
        const double d = r - cut.rsi;
        const double dp = d * d * (3.0 * c.sp_g3 + 4.0 * c.sp_g4 * d);
        const double dpp = d * (6.0 * c.sp_g3 + 12.0 * c.sp_g4 * d);
        fpair = -dp * ir;
        en = c.sp_g0 + d * d * d * (c.sp_g3 + d * c.sp_g4) - c.sp_shift;
        hc = (-dpp - fpair) * ir * ir;
    } else if (r2 < cut.rci2) {
        const double r2i = M::recip(r2);
        const double r6i = r2i * r2i * r2i;
        fpair = r6i * (c.cg_c12 * r6i - c.cg_c6) * r2i;
        en = r6i * (c.cg_e12 * r6i - c.cg_e6) - c.cm_shift;
        hc = r2i * r2i * r6i * (8.0 * c.cg_c6 - 14.0 * c.cg_c12 * r6i);
    } else {
        double r, ir;
        M::root(r2, r, ir);
        const double d = r - cut.rci;
        const double dp = c.cm_g[1] + d * (2.0 * c.cm_g[2] + d * (3.0 * c.cm_g[3] + d * (4.0 * c.cm_g[4])));
        const double dpp = 2.0 * c.cm_g[2] + d * (6.0 * c.cm_g[3] + d * (12.0 * c.cm_g[4]));
        fpair = -dp * ir;
        en = c.cm_g[0] + d * (c.cm_g[1] + d * (c.cm_g[2] + d * (c.cm_g[3] + d * c.cm_g[4]))) - c.cm_shift;
        hc = (-dpp - fpair) * ir * ir;
    }
}

// One list row of the backward pass (FG part when CG is false, CG part when
// true); TM bounds the number of types.
template <bool CG, int TM>
__device__ __forceinline__ void back_row(const BackArgs& b, const BoxV& bx, int ti,
                                         double xi, double yi, double zi, double gix, double giy,
                                         double giz, double ebar, const int* __restrict__ lst,
                                         int cnt, int sub, int G, double gp[3], double acc[TM][4])
{
    const ForceArgs& a = b.f;
    const int nt = a.ntypes;
    const int np = nt * nt;
    const PairCoef<double>* coef = (const PairCoef<double>*)a.coef64;
    constexpr int P0 = CG ? 2 : 0;
    for (int k = sub; k < cnt; k += G) {
        const uint32_t e = (uint32_t)lst[k];
        const int uj = (int)(e & kIdxMask), tj = (int)(e >> kIdxBits);
        double dx = xi - a.pos[3 * uj];
        double dy = yi - a.pos[3 * uj + 1];
        double dz = zi - a.pos[3 * uj + 2];
        dx -= bx.L[0] * rint(dx * bx.iL[0]);
        dy -= bx.L[1] * rint(dy * bx.iL[1]);
        dz -= bx.L[2] * rint(dz * bx.iL[2]);
        const double r2 = dx * dx + dy * dy + dz * dz;
        const int pi = ti * nt + tj;
        const Cutoffs<double>& cut = a.pcut64[pi];
        if (!(r2 < (CG ? cut.rco2 : cut.rso2))) continue;
        double fp, en, hc, fe, ee, fs, es;
        if constexpr (CG) {
            cg_terms2(coef[pi], cut, r2, fp, en, hc);
            cg_term<MathF64<2>>(b.cgrad[2 * np + pi], cut, r2, fe, ee);
            cg_term<MathF64<2>>(b.cgrad[3 * np + pi], cut, r2, fs, es);
        } else {
            fg_terms2(coef[pi], cut, r2, fp, en, hc);
            fg_term<MathF64<2>>(b.cgrad[0 * np + pi], cut, r2, fe, ee);
            fg_term<MathF64<2>>(b.cgrad[1 * np + pi], cut, r2, fs, es);
        }
        double wx = gix, wy = giy, wz = giz;
        if (b.gforce) {
            wx -= b.gforce[3 * uj];
            wy -= b.gforce[3 * uj + 1];
            wz -= b.gforce[3 * uj + 2];
        }
        const double dw = dx * wx + dy * wy + dz * wz;
        gp[0] += -ebar * fp * dx + fp * wx + hc * dw * dx;
        gp[1] += -ebar * fp * dy + fp * wy + hc * dw * dy;
        gp[2] += -ebar * fp * dz + fp * wz + hc * dw * dz;
        const double gd = gix * dx + giy * dy + giz * dz;
        const double ve = 0.5 * ebar * ee + gd * fe;
        const double vs = 0.5 * ebar * es + gd * fs;
#pragma unroll
        for (int q = 0; q < TM; ++q)
            if (q == tj) {
                acc[q][P0] += ve;
                acc[q][P0 + 1] += vs;
            }
    }
}

template <int TM>
__global__ __launch_bounds__(kForceBlock) void k_backward(BackArgs b)
{
    const ForceArgs& a = b.f;
    const bool rb = (int)blockIdx.x >= a.blocks_a;
    const int lb = rb ? (int)blockIdx.x - a.blocks_a : (int)blockIdx.x;
    const int nb = rb ? a.blocks_b : a.blocks_a;
    const int per = nb >> 3;
    const int logical = (lb & 7) * per + (lb >> 3);
    const int lg = rb ? a.log_lanes_b : a.log_lanes_a;
    const int G = 1 << lg;
    const int row = logical * (kForceBlock >> lg) + ((int)threadIdx.x >> lg);
    const int sub = (int)threadIdx.x & (G - 1);

    int4 rec = make_int4(-1, 0, 0, 1);
    int cnt_a = 0;
    if (!rb) {
        if (row < a.n_arow) rec = a.a_rec[row];
    } else if (row < a.n_srow) {
        rec = a.s_rec[row];
        cnt_a = a.a_rec[rec.w].z;
    }
    const bool own = rb ? rec.x >= 0 : (rec.x >= 0 && rec.w == 0);
    const int sy = rec.x >= 0 ? rec.y >> kTypeBits : 0;
    const double ebar = b.genergy ? b.genergy[sy] : 0.0;
    const BoxV bx = row_box(a, sy);
    double acc[TM][4];
#pragma unroll
    for (int q = 0; q < TM; ++q)
#pragma unroll
        for (int P = 0; P < 4; ++P) acc[q][P] = 0.0;
    double gp[3] = {0.0, 0.0, 0.0};
    const int ti = rec.y & ((1 << kTypeBits) - 1);
    if (own) {
        const int ui = rec.x;
        const double xi = a.pos[3 * ui], yi = a.pos[3 * ui + 1], zi = a.pos[3 * ui + 2];
        double gix = 0.0, giy = 0.0, giz = 0.0;
        if (b.gforce) {
            gix = b.gforce[3 * ui];
            giy = b.gforce[3 * ui + 1];
            giz = b.gforce[3 * ui + 2];
        }
        const int ar = rb ? rec.w : row;
        const int ca = rb ? cnt_a : rec.z;
        back_row<false, TM>(b, bx, ti, xi, yi, zi, gix, giy, giz, ebar,
                            a.a_list + (size_t)ar * a.a_cap, ca, sub, G, gp, acc);
        if (rb)
            back_row<true, TM>(b, bx, ti, xi, yi, zi, gix, giy, giz, ebar,
                               a.s_list + (size_t)row * a.s_cap, rec.z, sub, G, gp, acc);
    }
    for (int c = 0; c < 3; ++c) gp[c] = group_sum(gp[c], G);
    if (own && sub == 0) {
        b.gpos[3 * rec.x] = gp[0];
        b.gpos[3 * rec.x + 1] = gp[1];
        b.gpos[3 * rec.x + 2] = gp[2];
    }
    // per-wave sums per (row type, entry type, parameter), fixed order
    const int nt = a.ntypes;
    const int nbins = 4 * nt * nt;
    const int wave = (int)blockIdx.x * (kForceBlock / 64) + (int)(threadIdx.x >> 6);
    double* out = b.partial + (size_t)wave * nbins;
    for (int t = 0; t < nt; ++t)
#pragma unroll
        for (int q = 0; q < TM; ++q) {
            if (q >= nt) break;
            // the four parameters' sums at once (their chains interleaved)
            double s[4];
#pragma unroll
            for (int P = 0; P < 4; ++P) s[P] = (own && ti == t) ? acc[q][P] : 0.0;
            wave_sums(s);
            if ((threadIdx.x & 63) == 63) {
#pragma unroll
                for (int P = 0; P < 4; ++P) out[(t * nt + q) * 4 + P] = s[P];
            }
        }
}

// dJ/dP[a][b] = sum over waves of the partial sums, in wave order; one block
// per bin.
__global__ __launch_bounds__(256) void k_reduce_bins(const double* __restrict__ partial, int waves,
                                                     int nt, double* __restrict__ grad_pair)
{
    __shared__ double red[4];
    const int bin = (int)blockIdx.x;             // (t * nt + q) * 4 + P
    const int nbins = 4 * nt * nt;
    double s = 0.0;
    for (int w = (int)threadIdx.x; w < waves; w += 256) s += partial[(size_t)w * nbins + bin];
    const double v = wave_sum(s);
    if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int P = bin & 3, tq = bin >> 2;
        grad_pair[(size_t)P * nt * nt + tq] = red[0] + red[1] + red[2] + red[3];
    }
}

hipError_t launch_backward(const BackArgs& b, int waves, double* grad_pair, hipStream_t s)
{
    const int nt = b.f.ntypes;
    const int blocks = b.f.blocks_a + b.f.blocks_b;
    if (blocks > 0) {
        const dim3 grid(blocks), block(kForceBlock);
        if (nt <= 2)
            hipLaunchKernelGGL(k_backward<2>, grid, block, 0, s, b);
        else if (nt <= 4)
            hipLaunchKernelGGL(k_backward<4>, grid, block, 0, s, b);
        else
            hipLaunchKernelGGL(k_backward<8>, grid, block, 0, s, b);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_reduce_bins, dim3(4 * nt * nt), dim3(256), 0, s, b.partial,
                       blocks > 0 ? waves : 0, nt, grad_pair);
    return hipGetLastError();
}

// Chain rule from pair-table gradients to per-type parameters: for type t and
// family f (FG, CG), dJ/d eps_t = sum over ordered pairs (t, b) and (a, t) of
// dJ/d eps_ab times d eps_ab/d eps_t, and dJ/d sigma_t likewise through
// eps_ab and sigma_ab.  jac[(f * nt^2 + q) * 6] holds, for pair q = a*nt + b,
// the derivatives of (eps_ab, eps_ab, sigma_ab) with respect to (eps_a,
// sigma_a, sigma_a), then those with respect to type b's values.  One thread
// per output, sums in a fixed order.
__global__ __launch_bounds__(256) void k_type_grad(const double* __restrict__ gpair,
                                                   const double* __restrict__ jac, int nt,
                                                   double* __restrict__ gtype)
{
    const int o = (int)threadIdx.x;
    if (o >= 4 * nt) return;
    const int P = o / nt, t = o % nt;
    const int f = P >> 1, y = P & 1;          // family, 0 = eps / 1 = sigma
    const size_t np = (size_t)nt * nt;
    const double* ge = gpair + (size_t)(2 * f) * np;       // dJ/d eps_ab of the family
    const double* gs = gpair + (size_t)(2 * f + 1) * np;   // dJ/d sigma_ab
    const double* J = jac + (size_t)f * np * 6;
    double s = 0.0;
    for (int b = 0; b < nt; ++b) {            // pairs (t, b): type t is the first
        const size_t q = (size_t)t * nt + b;
        s += y == 0 ? ge[q] * J[6 * q] : ge[q] * J[6 * q + 1] + gs[q] * J[6 * q + 2];
    }
    for (int a = 0; a < nt; ++a) {            // pairs (a, t): type t is the second
        const size_t q = (size_t)a * nt + t;
        s += y == 0 ? ge[q] * J[6 * q + 3] : ge[q] * J[6 * q + 4] + gs[q] * J[6 * q + 5];
    }
    gtype[o] = s;
}

hipError_t launch_type_grad(const double* gpair, const double* jac, int nt, double* gtype,
                            hipStream_t s)
{
    hipLaunchKernelGGL(k_type_grad, dim3(1), dim3(256), 0, s, gpair, jac, nt, gtype);
    return hipGetLastError();
}

// Energy/virial scratch of relres_forces_noalloc, for callers that cannot
// allocate: the launch epoch in its first 256 bytes, then the block and group
// records of the force kernel.  One copy per GPU, zero at load, shared by
// every call on that GPU (calls that overlap on one GPU race).  Host code
// reaches it only through the address scratch_address() returns.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(void** out)
{
    return hipGetSymbolAddress(out, HIP_SYMBOL(scratch));
}

__global__ void k_clear_words(unsigned long long* p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

hipError_t launch_clear_words(unsigned long long* p, size_t n, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    size_t blocks = (n + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_clear_words, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_zero_outputs(double* energy, double* virial, int nsys, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_outputs, dim3(1), dim3(256), 0, s, energy, virial, nsys);
    return hipGetLastError();
}

hipError_t launch_reduce_sys_ew(const GridDev* grids_dev, int ngrids, const ForceArgs& a,
                                double* energy, double* virial, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_sys_ew, dim3(a.nsys), dim3(256), 0, s, grids_dev, ngrids, a,
                       energy, virial);
    return hipGetLastError();
}

}  // namespace relres

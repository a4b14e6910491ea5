// CDNA4 (gfx950) kernels of the CR-MC hot path.
//
//   k_bin        per sweep: draw the grid shift, re-bin every record into the
//                shifted cells (stable: old cell order, then order in the old
//                cell), sample per-site occupancy, publish the sweep's shift and
//                pairing table.  Each new cell gathers from the old cells that
//                overlap it (at most 27, usually 8), one or (on large launches)
//                eight cells per wavefront: places records without atomics or
//                a global scan.
//   k_plan       per sweep: sorts the domains of every colour into light ones
//                (one wavefront each) and heavy ones (a whole workgroup); with
//                the learned proposal on, lists the feature kernel's work items.
//   k_phase<R, L, M> per colour: every domain (one cell, or two reflection-paired
//                cells of the colour) runs its trials back to back: Philox
//                words ten trials at a time, move and participants, pair
//                sum of the energy change over the domain's own lists (LDS)
//                and its 26-cell neighbourhoods (staged in LDS once, the excess
//                read from memory), R = float or double terms with FP64
//                accumulation,
//                acceptance of Sec. II C, commit in LDS; writes the cells back
//                at the end.  L: the learned site proposal compiled in; M: the
//                ion relocation trials compiled in.  k_phase_fast<R, M>: the
//                same, with the trials of empty domains evaluated side by
//                side (batches with sparse replicas).
//   k_sweep_end  per sweep: folds the domains' counter stripes, series row,
//                group histograms, next grid shift;
//                k_sweep_advance then advances the sweep counter.
//   k_energy     total energy of a replica from scratch (FP64), per cell.
#include "crmc_internal.h"

#include <math.h>

#include <mutex>

namespace crmc {

// ------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// ------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t out[4])
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// ------------------------------------------------------------------------
// integer helpers
// ------------------------------------------------------------------------
__device__ __forceinline__ uint32_t pick32(uint32_t w, uint32_t m) { return __umulhi(w, m); }

__device__ __forceinline__ uint32_t pick64(uint32_t hi, uint32_t lo, uint32_t m)
{
    const uint64_t top = (uint64_t)hi * m + (uint64_t)__umulhi(lo, m);
    return (uint32_t)(top >> 32);
}

__device__ __forceinline__ double unit53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ uint32_t cell_of(uint32_t y, uint32_t n) { return __umulhi(y, n); }

__device__ __forceinline__ void grid_shift(uint32_t k0, uint32_t k1, uint64_t sweep, int fixed, uint32_t o[3])
{
    if (fixed) { o[0] = o[1] = o[2] = 0u; return; }
    uint32_t w[4];
    philox4x32_10((uint32_t)sweep, 0u, 0u, TAG_SHIFT, k0, k1, w);
    o[0] = w[0]; o[1] = w[1]; o[2] = w[2];
}

__device__ __forceinline__ int rec_kind(uint32_t meta) { return (int)(meta & 7u); }
__device__ __forceinline__ int rec_charged(uint32_t meta) { return (int)((meta >> 3) & 1u); }
__device__ __forceinline__ int rec_is_ion(uint32_t meta)
{
    const uint32_t k = meta & 7u;
    return k == KIND_XPOS || k == KIND_XNEG;
}
// Charge of a record from its kind and charged flag (meta & 15 = kind + 8
// charged), looked up branch-free: two bits per value hold q + 1.  An acid is
// -1 when charged, a base +1, a cation +1 and an anion -1 whatever the flag,
// everything else 0.  The second table gives free ions charge 0 (ions that do
// not couple).
constexpr uint32_t Q_TABLE = 0x54a15495u, Q_TABLE_NO_ION = 0x55615555u;
__device__ __forceinline__ int rec_q(uint32_t meta)
{
    return (int)((Q_TABLE >> (2u * (meta & 15u))) & 3u) - 1;
}

__device__ __forceinline__ uint32_t rdl0(uint32_t v) { return (uint32_t)__builtin_amdgcn_readlane((int)v, 0); }

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const uint32_t lane = threadIdx.x & 63u;
    return lane ? (~0ull >> (64u - lane)) : 0ull;
}

// ------------------------------------------------------------------------
// k_bin: stable re-binning into the shifted grid of this sweep
// ------------------------------------------------------------------------
// grid shifts of this sweep (on) and of the previous one (oo)
__device__ __forceinline__ void bin_shifts(const Replica& R, uint64_t s, int fixed_grid, uint32_t on[3], uint32_t oo[3])
{
    if (R.tab->valid == s + 1u) {
        // left by the end of the previous sweep
        for (int d = 0; d < 3; ++d) { on[d] = R.tab->next[d]; oo[d] = R.tab->prev[d]; }
    } else {
        grid_shift(R.key0, R.key1, s, fixed_grid, on);
        if (s == 0) { oo[0] = oo[1] = oo[2] = 0u; }
        else grid_shift(R.key0, R.key1, s - 1, fixed_grid, oo);
    }
}

// the old cells that overlap new cell kc, per dimension in ascending order
__device__ __forceinline__ void bin_candidates(const uint32_t* __restrict__ bnd, uint32_t n, const uint32_t kc[3],
                                               const uint32_t on[3], const uint32_t oo[3], uint32_t cand[3][3],
                                               int ncand[3])
{
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const uint32_t lo_abs = on[d] + bnd[kc[d]];
        const uint32_t hi_abs = on[d] + bnd[kc[d] + 1] - 1u;
        const uint32_t j0 = cell_of(lo_abs - oo[d], n), j1 = cell_of(hi_abs - oo[d], n);
        const int m = (int)((j1 + n - j0) % n) + 1;
        uint32_t v0 = j0, v1 = (j0 + 1u) % n, v2 = (j0 + 2u) % n;
        // ascending order (a wrap-around puts small indices last)
        if (m == 2 && v1 < v0) { uint32_t t = v0; v0 = v1; v1 = t; }
        if (m == 3) {
            if (v1 < v0) { uint32_t t = v0; v0 = v1; v1 = t; }
            if (v2 < v1) { uint32_t t = v1; v1 = v2; v2 = t; }
            if (v1 < v0) { uint32_t t = v0; v0 = v1; v1 = t; }
        }
        cand[d][0] = v0; cand[d][1] = v1; cand[d][2] = v2;
        ncand[d] = m;
    }
}

// What the re-binning of one replica in one sweep needs (wavefront-uniform)
struct BinRep {
    uint64_t s;
    const uint4* src;
    const uint32_t* scnt;
    uint4* dst;
    uint32_t n, cap, hw, nxt;
    uint32_t on[3], oo[3];
};

__device__ __forceinline__ void bin_rep(const SweepArgs& a, const Replica& R, BinRep& b)
{
    b.s = *a.sweep;
    const int cur = (int)(b.s & 1u);
    b.nxt = (uint32_t)(cur ^ 1);
    b.src = R.rec[cur];
    b.scnt = R.cnt[cur];
    b.dst = R.rec[b.nxt];
    b.n = R.n;
    b.cap = R.cap;
    b.hw = *R.hiwater;
    bin_shifts(R, b.s, a.fixed_grid, b.on, b.oo);
}

// the sweep's table of a replica (its cell 0's duty): shift, and the
// pairing centre of every colour
__device__ __forceinline__ void bin_table(const Replica& R, const BinRep& b, uint32_t lane)
{
    if (lane < 12) {
        const uint32_t M = R.h * R.h * R.h;
        uint32_t v = 0;
        if (lane < 4) v = lane == 0 ? b.on[0] : (lane == 1 ? b.on[1] : (lane == 2 ? b.on[2] : 0u));
        else {
            uint32_t w[4];
            philox4x32_10((uint32_t)b.s, lane - 4u, 0u, TAG_PAIR, R.key0, R.key1, w);
            const uint32_t rr = pick32(w[0], M);
            v = (uint32_t)(((uint64_t)M - 1u + 2ull * M - 2ull * rr) % M);
        }
        if (lane < 4) R.tab->o[lane] = v; else R.tab->pairc[lane - 4] = v;
    }
}

// One chunk of candidate records (one per lane) for new cell k: the matches
// are appended in order after `base` (stable), sites counted, and every
// charged site sampled into its occupancy and its group's counter
__device__ __forceinline__ void bin_take(const Replica& R, const BinRep& b, uint32_t k, const uint32_t kc[3], bool valid,
                                         const uint4& rec, uint32_t lane, uint32_t& base, uint32_t& nsite)
{
    const uint32_t n = b.n;
    const bool match = valid && cell_of(rec.x - b.on[0], n) == kc[0] && cell_of(rec.y - b.on[1], n) == kc[1] &&
                       cell_of(rec.z - b.on[2], n) == kc[2];
    const uint64_t mask = __ballot(match);
    const uint32_t kd = rec.w & 7u;
    nsite += (uint32_t)__popcll(__ballot(match && (kd == KIND_ACID || kd == KIND_BASE)));
    const uint32_t sid = rec.w >> 8;
    const bool charged_site = match && sid != NO_SITE && rec_charged(rec.w);
    int grp = -1;
    if (match) {
        const uint32_t pos = base + (uint32_t)__popcll(mask & lanemask_lt());
        if (pos < b.cap) b.dst[(size_t)k * b.cap + pos] = rec;
        // each site lands in exactly one new cell: non-returning adds
        if (charged_site) {
            atomicAdd((unsigned long long*)&R.occupancy[sid], 1ull);
            grp = R.site_group[sid];
        }
    }
    // the group counters take one add per group present (a cell's sites
    // mostly share one group, and thousands of cells share each counter)
    uint64_t pend = __ballot(charged_site);
    while (pend) {
        const int lead = (int)__builtin_ctzll(pend);
        const int g = __builtin_amdgcn_readlane(grp, lead);
        const uint64_t same = __ballot(grp == g) & pend;
        if ((int)lane == lead) atomicAdd(&R.group_count[(b.s & 1u) * R.ngroups + (uint32_t)g], (int)__popcll(same));
        pend &= ~same;
    }
    base += (uint32_t)__popcll(mask);
}

__device__ __forceinline__ void bin_finish(const SweepArgs& a, const Replica& R, const BinRep& b, uint32_t k,
                                           uint32_t base, uint32_t nsite, uint32_t lane)
{
    if (lane == 0) {
        R.cnt[b.nxt][k] = base < b.cap ? base : b.cap;
        R.cnt0[k] = base < b.cap ? base : b.cap;
        R.nsc[k] = nsite;
        if (base > b.cap) atomicOr(a.err, ERR_BIN_CAPACITY);
        if (base > b.hw) atomicMax(R.hiwater, base); // rarely taken once the mark has settled
    }
}

// New cell k by the whole wavefront, for any number of candidate cells and
// any list length: the overlapping old cells in ascending (z, y, x) order,
// one per lane, with their counts loaded at once and scanned
__device__ void bin_cell(const SweepArgs& a, const Replica& R, const BinRep& b, uint32_t k, uint32_t lane)
{
    const uint32_t n = b.n, cap = b.cap;
    const uint32_t kc[3] = {k % n, (k / n) % n, k / (n * n)};
    uint32_t cand[3][3];
    int ncand[3];
    bin_candidates(R.bnd, n, kc, b.on, b.oo, cand, ncand);
    const int nc0 = ncand[0], nc01 = ncand[0] * ncand[1], ncand_all = nc01 * ncand[2];
    uint32_t my_oc = 0, my_cc = 0;
    if ((int)lane < ncand_all) {
        const int ix = (int)lane % nc0, iy = ((int)lane / nc0) % ncand[1], iz = (int)lane / nc01;
        const uint32_t cx = ix == 0 ? cand[0][0] : (ix == 1 ? cand[0][1] : cand[0][2]);
        const uint32_t cy = iy == 0 ? cand[1][0] : (iy == 1 ? cand[1][1] : cand[1][2]);
        const uint32_t cz = iz == 0 ? cand[2][0] : (iz == 1 ? cand[2][1] : cand[2][2]);
        my_oc = cx + n * (cy + n * cz);
        my_cc = b.scnt[my_oc];
    }
    uint32_t incl = my_cc;
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) {
        const uint32_t v = (uint32_t)__shfl_up((int)incl, off, 64);
        if ((int)lane >= off) incl += v;
    }
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, ncand_all - 1);
    uint32_t base = 0, nsite = 0;
    if (total <= 64u) {
        // lane j takes record j of the concatenated lists
        uint32_t oc = 0, idx = 0;
        for (int c = 0; c < ncand_all; ++c) {
            const uint32_t end = (uint32_t)__builtin_amdgcn_readlane((int)incl, c);
            const uint32_t cc = (uint32_t)__builtin_amdgcn_readlane((int)my_cc, c);
            const uint32_t occ = (uint32_t)__builtin_amdgcn_readlane((int)my_oc, c);
            if (lane >= end - cc && lane < end) { oc = occ; idx = lane - (end - cc); }
        }
        uint4 rec = make_uint4(0, 0, 0, 0);
        if (lane < total) rec = b.src[(size_t)oc * cap + idx];
        bin_take(R, b, k, kc, lane < total, rec, lane, base, nsite);
    } else {
        for (int c = 0; c < ncand_all; ++c) {
            const uint32_t oc = (uint32_t)__builtin_amdgcn_readlane((int)my_oc, c);
            const uint32_t cc = (uint32_t)__builtin_amdgcn_readlane((int)my_cc, c);
            for (uint32_t b0 = 0; b0 < cc; b0 += 64u) {
                const uint32_t i = b0 + lane;
                uint4 rec = make_uint4(0, 0, 0, 0);
                if (i < cc) rec = b.src[(size_t)oc * cap + i];
                bin_take(R, b, k, kc, i < cc, rec, lane, base, nsite);
            }
        }
    }
    bin_finish(a, R, b, k, base, nsite, lane);
}

// One wavefront per bin_cpw (1 or BIN_CPW) consecutive new cells of the
// dense replicas; the cells of sparse replicas (far fewer records than
// cells) are left to k_bin_sparse.  The cell index is uniform over the wavefront, so the
// replica, its tables and the grid shifts come through scalar loads.  The
// cells of one replica whose candidates are at most eight old cells holding
// at most 64 records in all (the common case) are re-binned together: lane
// 8i + c holds candidate c of cell i, so the counts of all of them arrive in
// one load, and the records of all of them (one per lane and cell) in one
// round; the others go one by one through bin_cell.  Every cell gets the
// same stable order either way.
__global__ __launch_bounds__(BIN_THREADS) void k_bin(SweepArgs a)
{
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63u;
    const uint32_t cpw = (uint32_t)a.bin_cpw;
    const uint32_t g0 = (blockIdx.x * (BIN_THREADS / 64) + wave) * cpw;
    if (g0 >= a.ncell_total) return;
    // a replica's cell count (an even edge count, cubed) is a multiple of
    // BIN_CPW, so the cells of a wavefront belong to one replica
    const uint32_t gend = min(g0 + cpw, a.ncell_total);
    const uint32_t r = a.cell2rep[g0];
    const Replica& R = a.reps[r];
    if (g0 == 0 && lane < 24 && !R.bin_sparse)
        a.plan_n[plan_idx(lane / 3, lane % 3)] = 0u; // plan and learned-proposal counters of the sweep
    if (R.bin_sparse) return;
    BinRep b;
    bin_rep(a, R, b);
    const uint32_t n = b.n, cap = b.cap;
    const uint32_t k0 = g0 - R.cell_begin, m = gend - g0;
    if (k0 == 0) bin_table(R, b, lane);
    if (cpw == 1) {
        bin_cell(a, R, b, k0, lane);
        return;
    }

    // lane 8i + c: candidate c of cell k0 + i
    const uint32_t ci = lane >> 3, cs = lane & 7u;
    const bool live = ci < m;
    const uint32_t k = k0 + (live ? ci : 0u);
    const uint32_t kc[3] = {k % n, (k / n) % n, k / (n * n)};
    uint32_t cand[3][3];
    int ncand[3];
    bin_candidates(R.bnd, n, kc, b.on, b.oo, cand, ncand);
    const int nc0 = ncand[0], nc01 = ncand[0] * ncand[1], ncand_all = nc01 * ncand[2];
    const bool few = ncand_all <= 8;
    uint32_t my_oc = 0, my_cc = 0;
    if (live && few && (int)cs < ncand_all) {
        const int ix = (int)cs % nc0, iy = ((int)cs / nc0) % ncand[1], iz = (int)cs / nc01;
        const uint32_t cx = ix == 0 ? cand[0][0] : (ix == 1 ? cand[0][1] : cand[0][2]);
        const uint32_t cy = iy == 0 ? cand[1][0] : (iy == 1 ? cand[1][1] : cand[1][2]);
        const uint32_t cz = iz == 0 ? cand[2][0] : (iz == 1 ? cand[2][1] : cand[2][2]);
        my_oc = cx + n * (cy + n * cz);
        my_cc = b.scnt[my_oc];
    }
    // inclusive scan of the counts within each group of eight lanes
    uint32_t incl = my_cc;
#pragma unroll
    for (int off = 1; off < 8; off <<= 1) {
        const uint32_t v = (uint32_t)__shfl_up((int)incl, off, 8);
        if ((int)cs >= off) incl += v;
    }
    const uint32_t tot = (uint32_t)__shfl((int)incl, (int)(lane | 7u), 64);
    // cells left to bin_cell: more than eight candidates or 64 records
    const uint64_t slow = __ballot(live && cs == 0 && (!few || tot > 64u));

    uint4 v[BIN_CPW];
#pragma unroll
    for (uint32_t i = 0; i < BIN_CPW; ++i) {
        v[i] = make_uint4(0u, 0u, 0u, 0u);
        if (i < m && !((slow >> (8 * i)) & 1ull)) {
            const uint32_t ti = (uint32_t)__builtin_amdgcn_readlane((int)tot, (int)(8 * i));
            uint32_t oc = 0, idx = 0;
#pragma unroll
            for (uint32_t c = 0; c < 8; ++c) {
                const uint32_t end = (uint32_t)__builtin_amdgcn_readlane((int)incl, (int)(8 * i + c));
                const uint32_t cc = (uint32_t)__builtin_amdgcn_readlane((int)my_cc, (int)(8 * i + c));
                const uint32_t occ = (uint32_t)__builtin_amdgcn_readlane((int)my_oc, (int)(8 * i + c));
                if (lane >= end - cc && lane < end) { oc = occ; idx = lane - (end - cc); }
            }
            if (lane < ti) v[i] = b.src[(size_t)oc * cap + idx];
        }
    }
#pragma unroll
    for (uint32_t i = 0; i < BIN_CPW; ++i) {
        if (i < m && !((slow >> (8 * i)) & 1ull)) {
            const uint32_t ti = (uint32_t)__builtin_amdgcn_readlane((int)tot, (int)(8 * i));
            const uint32_t kci[3] = {(uint32_t)__builtin_amdgcn_readlane((int)kc[0], (int)(8 * i)),
                                     (uint32_t)__builtin_amdgcn_readlane((int)kc[1], (int)(8 * i)),
                                     (uint32_t)__builtin_amdgcn_readlane((int)kc[2], (int)(8 * i))};
            uint32_t base = 0, nsite = 0;
            bin_take(R, b, k0 + i, kci, lane < ti, v[i], lane, base, nsite);
            bin_finish(a, R, b, k0 + i, base, nsite, lane);
        }
    }
    for (uint32_t i = 0; i < m; ++i)
        if ((slow >> (8 * i)) & 1ull) bin_cell(a, R, b, k0 + i, lane);
}

// One lane per new cell of the sparse replicas: the lane walks the
// overlapping old cells in the same order as k_bin and appends its matches
// one by one, so the result is the same stable order; 64 cells are in flight
// per wavefront instead of one.
__global__ __launch_bounds__(BIN_THREADS) void k_bin_sparse(SweepArgs a)
{
    const uint32_t gcell = blockIdx.x * BIN_THREADS + threadIdx.x;
    if (gcell >= a.ncell_total) return;
    const uint32_t r = a.cell2rep[gcell];
    const Replica& R = a.reps[r];
    if (!R.bin_sparse) return;
    const uint32_t n = R.n, cap = R.cap;
    const uint32_t k = gcell - R.cell_begin;
    const uint64_t s = *a.sweep;
    const int cur = (int)(s & 1u), nxt = cur ^ 1;
    const uint4* __restrict__ src = R.rec[cur];
    const uint32_t* __restrict__ scnt = R.cnt[cur];
    uint4* __restrict__ dst = R.rec[nxt];
    uint32_t on[3], oo[3];
    bin_shifts(R, s, a.fixed_grid, on, oo);
    // the duties of k_bin for the cells it leaves to this kernel: the sweep's
    // plan counters (with global cell 0) and the replica's table (with its cell 0)
    if (gcell == 0)
        for (int c = 0; c < 8; ++c)
            for (int j = 0; j < 3; ++j) a.plan_n[plan_idx(c, j)] = 0u;
    if (k == 0) {
        const uint32_t M = R.h * R.h * R.h;
        for (int d = 0; d < 3; ++d) R.tab->o[d] = on[d];
        R.tab->o[3] = 0u;
        for (uint32_t c = 0; c < 8u; ++c) {
            uint32_t w[4];
            philox4x32_10((uint32_t)s, c, 0u, TAG_PAIR, R.key0, R.key1, w);
            const uint32_t rr = pick32(w[0], M);
            R.tab->pairc[c] = (uint32_t)(((uint64_t)M - 1u + 2ull * M - 2ull * rr) % M);
        }
    }
    const uint32_t kc[3] = {k % n, (k / n) % n, k / (n * n)};
    uint32_t cand[3][3];
    int ncand[3];
    bin_candidates(R.bnd, n, kc, on, oo, cand, ncand);

    uint32_t base = 0, nsite = 0;
    // the lane's adds to one group counter are gathered while the group stays
    // the same (a chain's sites share one) and flushed when it changes
    int run_g = -1, run_n = 0;
    int32_t* gcnt = R.group_count + (s & 1u) * R.ngroups;
    for (int iz = 0; iz < ncand[2]; ++iz)
        for (int iy = 0; iy < ncand[1]; ++iy)
            for (int ix = 0; ix < ncand[0]; ++ix) {
                const uint32_t oc = cand[0][ix] + n * (cand[1][iy] + n * cand[2][iz]);
                const uint32_t cc = scnt[oc];
                for (uint32_t i = 0; i < cc; ++i) {
                    const uint4 rec = src[(size_t)oc * cap + i];
                    if (cell_of(rec.x - on[0], n) != kc[0] || cell_of(rec.y - on[1], n) != kc[1] ||
                        cell_of(rec.z - on[2], n) != kc[2])
                        continue;
                    if (base < cap) dst[(size_t)k * cap + base] = rec;
                    const uint32_t kd = rec.w & 7u;
                    nsite += (kd == KIND_ACID || kd == KIND_BASE) ? 1u : 0u;
                    const uint32_t sid = rec.w >> 8;
                    if (sid != NO_SITE && rec_charged(rec.w)) {
                        atomicAdd((unsigned long long*)&R.occupancy[sid], 1ull);
                        const int g = R.site_group[sid];
                        if (g != run_g) {
                            if (run_n) atomicAdd(&gcnt[run_g], run_n);
                            run_g = g;
                            run_n = 0;
                        }
                        ++run_n;
                    }
                    ++base;
                }
            }
    if (run_n) atomicAdd(&gcnt[run_g], run_n);
    R.cnt[nxt][k] = base < cap ? base : cap;
    R.cnt0[k] = base < cap ? base : cap;
    R.nsc[k] = nsite;
    if (base > cap) atomicOr(a.err, ERR_BIN_CAPACITY);
    if (base > *R.hiwater) atomicMax(R.hiwater, base);
}

// ------------------------------------------------------------------------
// precision policy of the pair terms
// ------------------------------------------------------------------------
template <typename Real> struct Math;
template <> struct Math<float> {
    // the hardware approximations (about 1 ulp; r^2 >= 1/4 wherever they matter)
    __device__ static __forceinline__ float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
    __device__ static __forceinline__ float ex(float x) { return __expf(x); }
    __device__ static __forceinline__ float ex2(float x) { return __builtin_amdgcn_exp2f(x); }
    __device__ static __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    __device__ static __forceinline__ float sqrt_(float x) { return sqrtf(x); }
};
template <> struct Math<double> {
    __device__ static __forceinline__ double rsqrt(double x) { return 1.0 / sqrt(x); }
    __device__ static __forceinline__ double ex(double x) { return exp(x); }
    __device__ static __forceinline__ double ex2(double x) { return exp2(x); }
    __device__ static __forceinline__ double rcp(double x) { return 1.0 / x; }
    __device__ static __forceinline__ double sqrt_(double x) { return sqrt(x); }
};

// ------------------------------------------------------------------------
// k_plan and k_phase: one colour of one sweep
// ------------------------------------------------------------------------
// A domain is one active cell, or two reflection-paired active cells of the
// colour.  The planning kernel (once per sweep, after the re-binning) sorts the
// domains of every colour into two lists: light domains run one per wavefront
// (four per workgroup, each with a quarter of the LDS pool), heavy ones
// (nanoparticle surfaces) get a whole workgroup.  A domain's own cells change
// only in its own phase, so the binned counts the plan uses size its pool
// exactly; its neighbour cells may have changed in earlier phases, which only
// changes how many neighbour records fit on chip.
constexpr int MAX_LDS_CORES = 64; // nanoparticle cores copied on chip (more are read from memory)

// LDS pool of one domain, offsets in 16-byte records:
//   member 0's list | member 1's list | ln k table (doubles) | cores | core
//   Deltas (doubles) | neighbour records (as many as fit)
// longest list (with room for growth) a light domain holds in registers, and
// the plan's flag for such a domain (a bit of the replica word of its slot)
constexpr int REG_ROOM = 64;
constexpr uint32_t GEO_REG = 0x80000000u;

struct Pool {
    int room0, room1;
    int ln_off, nln;
    int core_off, cdel_off, ncl;
    int aux_off;   // learned proposal: site probability per list slot (doubles)
    int st_off;
    __device__ __forceinline__ int base(int member) const { return member ? room0 : 0; }
};

__device__ __forceinline__ Pool pool_layout(int n0, int n1, int ncell, int ntr_max, uint32_t cap, uint32_t ncores,
                                            int learned)
{
    Pool p;
    // room for the growth the trials can cause: two ions per trial
    p.room0 = min((int)cap, n0 + 2 * ntr_max);
    p.room1 = ncell == 2 ? min((int)cap, n1 + 2 * ntr_max) : 0;
    p.ln_off = p.room0 + p.room1;
    p.nln = p.room0 + p.room1 + 2; // ln k for every count the domain can reach
    p.core_off = p.ln_off + (p.nln + 1) / 2;
    p.ncl = ncores <= (uint32_t)MAX_LDS_CORES ? (int)ncores : 0;
    p.cdel_off = p.core_off + p.ncl;
    p.aux_off = p.cdel_off + (p.ncl + 1) / 2;
    // the learned proposal's per-slot p_i (doubles), or with register lists its
    // eight class weights (at least four records either way)
    p.st_off = p.aux_off + (learned ? max((p.room0 + p.room1 + 1) / 2, 4) : 0);
    return p;
}

struct DomGeo {
    uint32_t cell0, cell1;
    uint32_t cc0[3], cc1[3];
    int ncell;
};

// active cells of domain d (0-based within the replica) in a colour
__device__ __forceinline__ DomGeo domain_geometry(const Replica& R, uint32_t d, int colour, int pairing)
{
    const uint32_t n = R.n, h = R.h, M = h * h * h;
    const uint32_t px = colour & 1, py = (colour >> 1) & 1, pz = (colour >> 2) & 1;
    uint32_t ma, mb;
    if (pairing) {
        const uint32_t c = R.tab->pairc[colour];
        const uint32_t half = c >> 1;
        if (d <= half) { ma = d; mb = c - d; }
        else { ma = c + 1u + (d - half - 1u); mb = M + c - ma; }
    } else {
        ma = mb = d;
    }
    DomGeo g;
    g.ncell = (ma == mb) ? 1 : 2;
    g.cc0[0] = 2u * (ma % h) + px; g.cc0[1] = 2u * ((ma / h) % h) + py; g.cc0[2] = 2u * (ma / (h * h)) + pz;
    g.cc1[0] = 2u * (mb % h) + px; g.cc1[1] = 2u * ((mb / h) % h) + py; g.cc1[2] = 2u * (mb / (h * h)) + pz;
    g.cell0 = g.cc0[0] + n * (g.cc0[1] + n * g.cc0[2]);
    g.cell1 = g.cc1[0] + n * (g.cc1[1] + n * g.cc1[2]);
    return g;
}

// neighbour o (0..25, the 3x3x3 block without its centre) of cell (x, y, z)
__device__ __forceinline__ uint32_t neighbour_cell(uint32_t x, uint32_t y, uint32_t z, int o, uint32_t n)
{
    const int oo = o < 13 ? o : o + 1;
    const uint32_t nx = (x + n + (uint32_t)(oo % 3) - 1u) % n;
    const uint32_t ny = (y + n + (uint32_t)((oo / 3) % 3) - 1u) % n;
    const uint32_t nz = (z + n + (uint32_t)(oo / 9) - 1u) % n;
    return nx + n * (ny + n * nz);
}

// one thread per domain, one colour per workgroup (blockIdx.y); the list
// slots are claimed with one atomic per wavefront and class, on a line of
// counters per colour (the colours' workgroups run side by side).  With the
// learned proposal on, each cell of the domain also gets its work items for
// the feature kernel: one per 64 sites (sites never change cells within a
// sweep, so the counts of the re-binning hold for all phases).
__global__ __launch_bounds__(64) void k_plan(SweepArgs a)
{
    const int colour = (int)blockIdx.y;
    const uint32_t gd = blockIdx.x * 64u + threadIdx.x;
    bool valid = gd < a.ndom_total, light = false;
    uint4 geo = make_uint4(0u, 0u, 0u, 0u);
    const auto plan_domain = [&](const Replica& R, uint32_t r) {
        const DomGeo G = domain_geometry(R, gd - R.dom_begin, colour, a.pairing);
        if (a.lwork) {
            for (int c = 0; c < G.ncell; ++c) {
                const uint32_t cell = c ? G.cell1 : G.cell0;
                const uint32_t m = (R.nsc[cell] + 63u) / 64u;
                if (m == 0u) continue;
                // the capacity bounds every sweep's items (sites / 64 + cells with sites)
                const uint32_t b = atomicAdd(&a.plan_n[plan_idx(colour, PLAN_LWORK)], m);
                const int buf = (int)((*a.sweep + 1u) & 1u);
                for (uint32_t i = 0; i < m && b + i < a.lwork_cap; ++i) {
                    LearnItem& L = a.lwork[(size_t)colour * a.lwork_cap + b + i];
                    L.rec = R.rec[buf];
                    L.cnt = R.cnt[buf];
                    L.phat = R.phat;
                    L.feat = R.feat;
                    L.off[0] = R.lp_off[0];
                    L.off[1] = R.lp_off[1];
                    L.cell = cell;
                    L.part = i;
                    L.r = r;
                    L.n = R.n;
                    L.cap = R.cap;
                    L.pad = 0;
                }
            }
        }
        const uint32_t* cntb = R.cnt[(*a.sweep + 1u) & 1u];
        int nb = 0;
#pragma unroll
        for (int o = 0; o < 26; ++o) nb += (int)cntb[neighbour_cell(G.cc0[0], G.cc0[1], G.cc0[2], o, R.n)];
        if (G.ncell == 2) {
#pragma unroll
            for (int o = 0; o < 26; ++o) nb += (int)cntb[neighbour_cell(G.cc1[0], G.cc1[1], G.cc1[2], o, R.n)];
        }
        const int n0 = (int)R.cnt0[G.cell0];
        const int n1 = G.ncell == 2 ? (int)R.cnt0[G.cell1] : 0;
        const int ntr_max = (a.trials + a.ion_trials) * G.ncell + ((n0 + n1) * a.site_trials + 15) / 16;
        const Pool p = pool_layout(n0, n1, G.ncell, ntr_max, R.cap, R.ncores, a.learned);
        light = nb <= a.light_nb && p.st_off <= a.pool / 4;
        // a light domain whose lists (with their room) fit 64 records each
        // keeps them in registers, one record per lane (flag: bit 31)
        const uint32_t reg = light && p.room0 <= REG_ROOM && p.room1 <= REG_ROOM ? GEO_REG : 0u;
        geo = make_uint4(r | reg, G.cell0, G.ncell == 2 ? G.cell1 : G.cell0, (uint32_t)n0 | ((uint32_t)n1 << 16));
    };
    // lane 0's domain is valid whenever any lane's is; when all the
    // wavefront's domains belong to one replica (the common case), its
    // descriptor and tables come through scalar loads
    const uint32_t r = a.dom2rep[valid ? gd : blockIdx.x * 64u];
    const uint32_t r0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)r);
    if (__ballot(r != r0) == 0ull) {
        if (valid) plan_domain(a.reps[r0], r0);
    } else if (valid) {
        plan_domain(a.reps[r], r);
    }
    const uint64_t ml = __ballot(valid && light), mh = __ballot(valid && !light);
    const uint32_t lane = threadIdx.x;
    uint32_t bl = 0, bh = 0;
    if (lane == 0) {
        if (ml) bl = atomicAdd(&a.plan_n[plan_idx(colour, PLAN_LIGHT)], (uint32_t)__popcll(ml));
        if (mh) bh = atomicAdd(&a.plan_n[plan_idx(colour, PLAN_HEAVY)], (uint32_t)__popcll(mh));
    }
    bl = rdl0(bl);
    bh = rdl0(bh);
    if (!valid) return;
    const uint64_t lt = lanemask_lt();
    if (light) {
        const size_t slot = (size_t)colour * a.ndom_total + bl + (uint32_t)__popcll(ml & lt);
        a.plan_light[slot] = gd;
        a.plan_geo_light[slot] = geo;
    } else {
        const size_t slot = (size_t)colour * a.ndom_total + bh + (uint32_t)__popcll(mh & lt);
        a.plan_heavy[slot] = gd;
        a.plan_geo_heavy[slot] = geo;
    }
}

// a particle whose state the trial changes
struct Chg {
    uint32_t x, y, z;
    int dq;      // charge change seen by every other particle
    int dw;      // +1 inserted free ion, -1 deleted free ion, 0 otherwise
    int member;  // domain cell it lives in
    int own;     // index in that cell's list, -1 if inserted
    int q_old, q_new, ion, pres_old, pres_new;
};

struct PairParams {
    float scale_f, sc2_f, kl_f; // lattice unit, its square, -kappa log2(e)
    float rc2_f, band_f;        // rc^2; half-width of the exact-test band (with room for rounding)
    double scale_d, sc2_d, kl_d;
    uint64_t R2;
    double rc2_lo, rc2_hi; // rc^2 (1 -+ 1e-5): outside this band the float distance decides
    double lB, kappa, eps;
    int ion_coupling;
};

template <typename Real>
__device__ __forceinline__ Real scale_of(const PairParams& P)
{
    return sizeof(Real) == 4 ? (Real)P.scale_f : (Real)P.scale_d;
}
template <typename Real>
__device__ __forceinline__ Real sc2_of(const PairParams& P)
{
    return sizeof(Real) == 4 ? (Real)P.sc2_f : (Real)P.sc2_d;
}
template <typename Real>
__device__ __forceinline__ Real kl_of(const PairParams& P)
{
    return sizeof(Real) == 4 ? (Real)P.kl_f : (Real)P.kl_d;
}

// squared distance (sigma^2) of a lattice offset, and the screened Coulomb
// kernel exp(-kappa r) / r from it
template <typename Real>
__device__ __forceinline__ Real r2_of(int32_t dx, int32_t dy, int32_t dz, const PairParams& P)
{
    const Real fx = (Real)dx, fy = (Real)dy, fz = (Real)dz;
    return (fx * fx + fy * fy + fz * fz) * sc2_of<Real>(P);
}
template <typename Real>
__device__ __forceinline__ Real yukawa(Real r2, const PairParams& P)
{
    const Real rinv = Math<Real>::rsqrt(r2);
    return Math<Real>::ex2(kl_of<Real>(P) * (r2 * rinv)) * rinv;
}

// The charge a record shows the Coulomb sum, as FP32 bits (it replaces the
// meta word in the on-chip copy of a neighbour record): zero for a free ion
// when ions do not couple.  Without coupling no excluded-volume term is
// evaluated either, so nothing else of the meta word is needed.
__device__ __forceinline__ uint32_t charge_bits(uint32_t meta, int ion_coupling)
{
    const uint32_t tab = ion_coupling ? Q_TABLE : Q_TABLE_NO_ION;
    const int q = (int)((tab >> (2u * (meta & 15u))) & 3u) - 1;
    return __float_as_uint((float)q);
}

// Per-lane sums for one changed particle c: aq = sum of q_j phi(r) over the
// records inside the Coulomb cutoff (times lB dq at the end), aw = excluded
// volume change; ov set on an overlap created by an insertion.  code is the
// record's charge_bits; valid = 0 masks the lane out.  Branch-free on the
// common path (the 64 lanes diverge anyway).  A record within 1e-5 of rc
// (rare) is left out; gap keeps the least |r^2 - rc^2| seen, and when that is
// inside the band pair_band adds such records afterwards if their exact
// integer distance is inside the cutoff.  The excluded-volume term sits
// behind a wavefront-uniform test.
template <typename Real>
__device__ __forceinline__ void pair_acc(const uint4& rec, uint32_t code, bool valid, const Chg& c,
                                         const PairParams& P, double& aq, double& aw, int& ov, float& gap)
{
    const int32_t dx = (int32_t)(rec.x - c.x), dy = (int32_t)(rec.y - c.y), dz = (int32_t)(rec.z - c.z);
    const Real r2 = r2_of<Real>(dx, dy, dz, P);
    const bool coupled = valid;
    if (c.dq != 0) {
        const bool in = r2 < (Real)P.rc2_lo;
        gap = fminf(gap, coupled ? fabsf((float)r2 - P.rc2_f) : 3.0e38f);
        const Real qphi = (Real)__uint_as_float(code) * yukawa<Real>(r2, P);
        aq += (double)((in && coupled) ? qphi : (Real)0);
    }
    if (c.dw != 0) {
        const bool near = coupled && r2 < (Real)1.2599210498948731647672106;
        if (__ballot(near)) {
            const bool over = near && r2 < (Real)0.25;
            const Real ir2 = Math<Real>::rcp(r2);
            const Real ir6 = ir2 * ir2 * ir2;
            const Real w = (Real)4.0 * (Real)P.eps * (ir6 * ir6 - ir6) + (Real)P.eps;
            aw += (double)((near && !over) ? (Real)c.dw * w : (Real)0);
            if (over && c.dw > 0) ov = 1;
        }
    }
}

// the Coulomb term of a record in the band around rc, if its exact squared
// lattice distance is inside the cutoff
template <typename Real>
__device__ __forceinline__ void pair_band(const uint4& rec, uint32_t code, bool valid, const Chg& c,
                                          const PairParams& P, double& aq)
{
    if (c.dq == 0) return;
    const int32_t dx = (int32_t)(rec.x - c.x), dy = (int32_t)(rec.y - c.y), dz = (int32_t)(rec.z - c.z);
    const Real r2 = r2_of<Real>(dx, dy, dz, P);
    if (valid && !(r2 < (Real)P.rc2_lo) && r2 <= (Real)P.rc2_hi) {
        const uint32_t ax = (uint32_t)abs(dx), ay = (uint32_t)abs(dy), az = (uint32_t)abs(dz);
        if ((uint64_t)ax * ax + (uint64_t)ay * ay + (uint64_t)az * az < P.R2)
            aq += (double)((Real)__uint_as_float(code) * yukawa<Real>(r2, P));
    }
}

// The expanded excluded volume of an ion against a core, in FP64 whatever
// the pair precision: the shifted distance r - Delta cancels most of r near a
// large core (in FP32 r = 10 keeps about 1e-6 absolute, and sh^-12 would carry
// 12 times that relative error of sh into the energy change)
template <typename Real>
__device__ __forceinline__ double wca_core(const Chg& c, const uint4& cx, double delta, const PairParams& P, int& ov)
{
    const int32_t dx = (int32_t)(cx.x - c.x), dy = (int32_t)(cx.y - c.y), dz = (int32_t)(cx.z - c.z);
    const double sc = P.scale_d;
    const double fx = (double)dx * sc, fy = (double)dy * sc, fz = (double)dz * sc;
    const double r2 = fx * fx + fy * fy + fz * fz;
    // far from the core (most pairs): out of reach without the square root;
    // the margin keeps every pair that the test below could take
    const double reach = delta + 1.122462048309373;
    if (r2 > reach * reach * (1.0 + 1e-12)) return 0.0;
    const double r = sqrt(r2);
    const double sh = r - delta;
    if (!(sh < 1.122462048309373)) return 0.0;
    if (sh < 0.5) {
        if (c.dw > 0) ov = 1;
        return 0.0;
    }
    const double ir2 = 1.0 / (sh * sh);
    const double ir6 = ir2 * ir2 * ir2;
    return (double)c.dw * (4.0 * P.eps * (ir6 * ir6 - ir6) + P.eps);
}

// the pair formed or broken between the two changed particles
template <typename Real>
__device__ __forceinline__ double changed_pair(const Chg& A, const Chg& B, const PairParams& P, bool ev_on, int& ov)
{
    if (!P.ion_coupling && (A.ion || B.ion)) return 0.0;
    const int32_t dx = (int32_t)(B.x - A.x), dy = (int32_t)(B.y - A.y), dz = (int32_t)(B.z - A.z);
    const uint32_t ax = (uint32_t)abs(dx), ay = (uint32_t)abs(dy), az = (uint32_t)abs(dz);
    const uint64_t r2i = (uint64_t)ax * ax + (uint64_t)ay * ay + (uint64_t)az * az;
    const Real sc = scale_of<Real>(P);
    const Real fx = (Real)dx * sc, fy = (Real)dy * sc, fz = (Real)dz * sc;
    const Real r2 = fx * fx + fy * fy + fz * fz;
    double e = 0.0;
    const int dqq = A.q_new * B.q_new - A.q_old * B.q_old;
    if (dqq != 0 && r2i < P.R2) {
        const Real rinv = Math<Real>::rsqrt(r2);
        e += P.lB * (double)dqq * (double)(Math<Real>::ex(-(Real)P.kappa * r2 * rinv) * rinv);
    }
    const int any_ion = A.ion || B.ion;
    const int pn = ev_on && any_ion && A.pres_new && B.pres_new;
    const int po = ev_on && any_ion && A.pres_old && B.pres_old;
    if ((pn || po) && r2 < (Real)1.2599210498948731647672106) {
        if (r2 < (Real)0.25) {
            if (pn) ov = 1;
        } else {
            const Real ir2 = Math<Real>::rcp(r2);
            const Real ir6 = ir2 * ir2 * ir2;
            e += (double)(pn - po) * (double)((Real)4.0 * (Real)P.eps * (ir6 * ir6 - ir6) + (Real)P.eps);
        }
    }
    return e;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }

// v from another lane through a DPP pattern (both halves of a double)
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(uint32_t)lo);
}

// sum over the 64 lanes, returned in every lane: quad butterflies and row
// rotations (DPP) give each 16-lane row its sum, then the four row sums
__device__ __forceinline__ double wave_sum_dpp(double v)
{
    v += dpp_d<0xB1>(v);  // quad_perm(1,0,3,2)
    v += dpp_d<0x4E>(v);  // quad_perm(2,3,0,1)
    v += dpp_d<0x124>(v); // row_ror:4
    v += dpp_d<0x128>(v); // row_ror:8
    const long long b = __double_as_longlong(v);
    double r[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int lo = __builtin_amdgcn_readlane((int)(uint32_t)b, 16 * k);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 16 * k);
        r[k] = __longlong_as_double(((long long)hi << 32) | (long long)(uint32_t)lo);
    }
    return (r[0] + r[1]) + (r[2] + r[3]);
}
// the same for 32-bit integers (sums modulo 2^32), returned uniform
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false);
    return ((uint32_t)__builtin_amdgcn_readlane((int)v, 0) + (uint32_t)__builtin_amdgcn_readlane((int)v, 16)) +
           ((uint32_t)__builtin_amdgcn_readlane((int)v, 32) + (uint32_t)__builtin_amdgcn_readlane((int)v, 48));
}
__device__ __forceinline__ uint32_t rflu(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ uint32_t rdl(uint32_t v, int lane) { return (uint32_t)__builtin_amdgcn_readlane((int)v, lane); }
__device__ __forceinline__ double rfld(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(uint32_t)lo);
}
// uniform values computed on the vector unit go back to scalar registers
__device__ __forceinline__ void uniform_chg(Chg& c)
{
    c.x = rflu(c.x); c.y = rflu(c.y); c.z = rflu(c.z);
    c.dq = rfl(c.dq); c.dw = rfl(c.dw); c.member = rfl(c.member); c.own = rfl(c.own);
    c.q_old = rfl(c.q_old); c.q_new = rfl(c.q_new); c.ion = rfl(c.ion);
    c.pres_old = rfl(c.pres_old); c.pres_new = rfl(c.pres_new);
}

// u < exp(min(0, lnp)) in FP64, decided from the single-precision exponential
// unless u lies within 1e-4 (relative) of it: that estimate is off by a few
// 1e-6 at most, so only near-ties pay for the double-precision exp
__device__ __forceinline__ bool metropolis(double u, double lnp)
{
    if (!(lnp < 0.0)) return u < 1.0;
    const double e = (double)__expf((float)lnp);
    if (u < e * (1.0 - 1e-4)) return true;
    if (u > e * (1.0 + 1e-4)) return false;
    return u < exp(lnp);
}

// LDS written by one lane becomes visible to the other lanes of its wavefront
// in program order; this keeps the compiler from moving memory accesses across
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Neighbour slots: the 26 neighbour cells of member 0, then those of member
// 1, concatenated; pre_v (lane q) holds the end of segment q, cell_v its cell.
// For the 64 slots g0 + lane, the source cell and index inside it; q is a
// cursor over the segments that only moves forward (uniform).
__device__ __forceinline__ void chunk_src(int g0, int lane, int& q, int pre_v, uint32_t cell_v, uint32_t& cell, int& off)
{
    while (q < 52 && (int)rdl((uint32_t)pre_v, q) <= g0) ++q;
    const int g = g0 + lane;
    cell = 0u;
    off = 0;
    for (int qq = q; qq < 52; ++qq) {
        const int st = qq ? (int)rdl((uint32_t)pre_v, qq - 1) : 0;
        if (st >= g0 + 64) break;
        const int en = (int)rdl((uint32_t)pre_v, qq);
        if (g >= st && g < en) {
            cell = rdl(cell_v, qq);
            off = g - st;
        }
    }
}

struct MemberCounts {
    int a0, ac, b0, bc, xp, xn; // neutral / charged acids and bases, cations, anions
};

__device__ __forceinline__ MemberCounts rfl_counts(const MemberCounts& c)
{
    return MemberCounts{rfl(c.a0), rfl(c.ac), rfl(c.b0), rfl(c.bc), rfl(c.xp), rfl(c.xn)};
}

// count changes of an accepted move: A's member gets the site change (moves
// 0-3) or the cation (4, 5), B's member the ion
__device__ __forceinline__ void apply_counts(MemberCounts& c, int move, bool hasA, bool hasB)
{
    const int s = (move & 1) ? -1 : 1; // forward / insertion: +1
    const bool acid = move <= 1, base = move == 2 || move == 3, salt = move >= 4;
    c.a0 -= (hasA && acid) ? s : 0;
    c.ac += (hasA && acid) ? s : 0;
    c.b0 -= (hasA && base) ? s : 0;
    c.bc += (hasA && base) ? s : 0;
    c.xp += ((hasA && salt) || (hasB && acid)) ? s : 0;
    c.xn += (hasB && !acid) ? s : 0;
}

__device__ __forceinline__ MemberCounts count_member(const uint4* pool, int base, int nn, int lane)
{
    MemberCounts c{0, 0, 0, 0, 0, 0};
    for (int b0 = 0; b0 < nn; b0 += 64) {
        const int g = b0 + lane;
        const uint32_t m = g < nn ? pool[base + g].w : 0u;
        const int kd = rec_kind(m), ch = rec_charged(m);
        c.a0 += __popcll(__ballot(kd == (int)KIND_ACID && !ch));
        c.ac += __popcll(__ballot(kd == (int)KIND_ACID && ch));
        c.b0 += __popcll(__ballot(kd == (int)KIND_BASE && !ch));
        c.bc += __popcll(__ballot(kd == (int)KIND_BASE && ch));
        c.xp += __popcll(__ballot(kd == (int)KIND_XPOS));
        c.xn += __popcll(__ballot(kd == (int)KIND_XNEG));
    }
    return c;
}

// index (in one member's list) of the k-th record whose meta word has
// (meta & mask) == value
__device__ __forceinline__ int member_kth(const uint4* pool, int base, int nn, uint32_t mask, uint32_t value, int k,
                                          int lane)
{
    const uint64_t lt = lanemask_lt();
    for (int b0 = 0; b0 < nn; b0 += 64) {
        const int g = b0 + lane;
        const bool p = g < nn && (pool[base + g].w & mask) == value;
        const uint64_t m = __ballot(p);
        const int c = __popcll(m);
        if (k < c) {
            const uint64_t hit = __ballot(p && __popcll(m & lt) == k);
            return b0 + (int)__builtin_ctzll(hit);
        }
        k -= c;
    }
    return -1;
}

// Learned pick within one member's list: the first eligible slot (meta &
// mask == value) whose cumulative weight (p or 1 - p of the slot's site,
// from aux) exceeds target; the last eligible slot if rounding leaves none.
__device__ __forceinline__ int member_kth_weighted(const uint4* pool, const double* aux, int base, int nn, uint32_t mask,
                                                   uint32_t value, bool fwd, double target, int lane)
{
    double acc = 0.0;
    int last = -1;
    for (int b0 = 0; b0 < nn; b0 += 64) {
        const int g = b0 + lane;
        const bool el = g < nn && (pool[base + g].w & mask) == value;
        const double a = el ? aux[base + g] : 0.0;
        double c = el ? (fwd ? a : 1.0 - a) : 0.0;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const double v = __shfl_up(c, off, 64);
            if (lane >= off) c += v;
        }
        c += acc;
        const uint64_t hit = __ballot(el && c > target);
        if (hit) return b0 + (int)__builtin_ctzll(hit);
        const uint64_t em = __ballot(el);
        if (em) last = b0 + 63 - (int)__builtin_clzll(em);
        acc = __shfl(c, 63, 64);
    }
    return last;
}

// per member: sum of p over neutral acids, of 1 - p over charged acids, and
// the same for bases (the weights of the learned picks)
struct ClassW {
    double a0_0, a0_1, ac_0, ac_1, b0_0, b0_1, bc_0, bc_1;
};

__device__ __forceinline__ void class_sums(const uint4* pool, const double* aux, int base, int nn, int lane,
                                           double& a0, double& ac, double& b0, double& bc)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int b = lane; b < nn; b += 64) {
        const uint32_t m = pool[base + b].w;
        const double p = aux[base + b];
        const int kd = rec_kind(m), ch = rec_charged(m);
        if (kd == (int)KIND_ACID) { if (ch) s1 += 1.0 - p; else s0 += p; }
        if (kd == (int)KIND_BASE) { if (ch) s3 += 1.0 - p; else s2 += p; }
    }
    a0 = wave_sum_dpp(s0);
    ac = wave_sum_dpp(s1);
    b0 = wave_sum_dpp(s2);
    bc = wave_sum_dpp(s3);
}

// class of a participant: meta mask and value
constexpr uint32_t CLS_MASK_SITE = 0xFu, CLS_MASK_ION = 0x7u;

// ---- lists of a light domain held in registers: record i of a member's list
//      in lane i (rooms of at most 64 records, which the plan checks), with the
//      learned proposal's site probability of the slot beside it.  The helpers
//      give the results of their LDS counterparts above for such lists.

__device__ __forceinline__ uint4 lane_rec(const uint4& r, int i)
{
    return make_uint4(rdl(r.x, i), rdl(r.y, i), rdl(r.z, i), rdl(r.w, i));
}
__device__ __forceinline__ double lane_d(double v, int i)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)b, i);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), i);
    return __longlong_as_double(((long long)hi << 32) | (long long)(uint32_t)lo);
}

__device__ __forceinline__ MemberCounts count_reg(uint32_t meta, int nn, int lane)
{
    const uint32_t m = lane < nn ? meta : 0u;
    const int kd = rec_kind(m), ch = rec_charged(m);
    MemberCounts c;
    c.a0 = __popcll(__ballot(kd == (int)KIND_ACID && !ch));
    c.ac = __popcll(__ballot(kd == (int)KIND_ACID && ch));
    c.b0 = __popcll(__ballot(kd == (int)KIND_BASE && !ch));
    c.bc = __popcll(__ballot(kd == (int)KIND_BASE && ch));
    c.xp = __popcll(__ballot(kd == (int)KIND_XPOS));
    c.xn = __popcll(__ballot(kd == (int)KIND_XNEG));
    return c;
}

__device__ __forceinline__ int reg_kth(uint32_t meta, int nn, uint32_t mask, uint32_t value, int k, int lane)
{
    const bool p = lane < nn && (meta & mask) == value;
    const uint64_t m = __ballot(p);
    if (k >= __popcll(m)) return -1;
    const uint64_t hit = __ballot(p && __popcll(m & lanemask_lt()) == k);
    return (int)__builtin_ctzll(hit);
}

__device__ __forceinline__ int reg_kth_weighted(uint32_t meta, double pd, int nn, uint32_t mask, uint32_t value,
                                                bool fwd, double target, int lane)
{
    const bool el = lane < nn && (meta & mask) == value;
    const double a = el ? pd : 0.0;
    double c = el ? (fwd ? a : 1.0 - a) : 0.0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double v = __shfl_up(c, off, 64);
        if (lane >= off) c += v;
    }
    const double acc = 0.0;
    c += acc;
    const uint64_t hit = __ballot(el && c > target);
    if (hit) return (int)__builtin_ctzll(hit);
    const uint64_t em = __ballot(el);
    return em ? 63 - (int)__builtin_clzll(em) : -1;
}

__device__ __forceinline__ void class_sums_reg(uint32_t meta, double pd, int nn, int lane, double& a0, double& ac,
                                               double& b0, double& bc)
{
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (lane < nn) {
        const int kd = rec_kind(meta), ch = rec_charged(meta);
        if (kd == (int)KIND_ACID) { if (ch) s1 += 1.0 - pd; else s0 += pd; }
        if (kd == (int)KIND_BASE) { if (ch) s3 += 1.0 - pd; else s2 += pd; }
    }
    a0 = wave_sum_dpp(s0);
    ac = wave_sum_dpp(s1);
    b0 = wave_sum_dpp(s2);
    bc = wave_sum_dpp(s3);
}

// swap-remove slot i of a register list of nn records; append at slot nn
__device__ __forceinline__ void reg_remove(uint4& r, double& d, int i, int nn, int lane, bool learned)
{
    const uint4 last = lane_rec(r, nn - 1);
    const double dl = learned ? lane_d(d, nn - 1) : 0.0;
    if (lane == i) {
        r = last;
        if (learned) d = dl;
    }
}
__device__ __forceinline__ void reg_append(uint4& r, double& d, int nn, uint4 v, int lane)
{
    if (lane == nn) {
        r = v;
        d = 0.0;
    }
}
// The domain's trials.  WPD wavefronts share the pair sums (WPD = 1: light
// domain, no workgroup barriers; WPD = 4: heavy domain, the whole workgroup;
// uniform over the workgroup).  REGL: the domain's lists in registers (light
// domains whose lists fit), else in the pool.
template <typename Real, bool LEARNED, bool RELOC, bool FAST, int WPD, bool REGL>
__device__ __forceinline__ void run_domain(const SweepArgs& a, uint32_t gd, uint4 geo, uint4* __restrict__ pool,
                                           int pool_records, int wid, double (*red)[4], int (*ovf)[4])
{
    static_assert(!REGL || WPD == 1, "register lists are held by one wavefront");
    constexpr int wpd = WPD;
    constexpr bool REG = REGL;
    constexpr int nt = 64 * wpd;
    const int lane = threadIdx.x & 63;
    const int tid = wid * 64 + lane;
    const uint64_t t_start = a.trace ? wall_clock64() : 0;
    const uint32_t r = rflu(geo.x) & ~GEO_REG;
    const Replica& R = a.reps[r];
    const uint32_t n = R.n, cap = R.cap;
    const uint64_t s = *a.sweep;
    const int buf = (int)((s + 1u) & 1u);
    uint4* __restrict__ recb = R.rec[buf];
    uint32_t* __restrict__ cntb = R.cnt[buf];
    const uint32_t key0 = R.key0, key1 = R.key1;
    const uint32_t ncores = R.ncores;
    const uint4* __restrict__ core_g = R.core_x;
    const double* __restrict__ cdel_g = R.core_delta;
    const int colour = a.colour;
    // the domain's cells and their binned counts, left by the plan kernel
    DomGeo G;
    G.cell0 = rflu(geo.y);
    G.cell1 = rflu(geo.z);
    G.ncell = G.cell1 != G.cell0 ? 2 : 1;
    G.cc0[0] = G.cell0 % n; G.cc0[1] = (G.cell0 / n) % n; G.cc0[2] = G.cell0 / (n * n);
    G.cc1[0] = G.cell1 % n; G.cc1[1] = (G.cell1 / n) % n; G.cc1[2] = G.cell1 / (n * n);
    const int ncell = G.ncell;
    (void)colour;

    int n0 = (int)(rflu(geo.w) & 0xFFFFu);
    int n1 = (int)(rflu(geo.w) >> 16);
    const int ntr_max = (a.trials + a.ion_trials) * ncell + ((n0 + n1) * a.site_trials + 15) / 16;
    const Pool pl = pool_layout(n0, n1, ncell, ntr_max, cap, ncores, LEARNED ? 1 : 0);
    // the plan and the host size pools (and light domains' lists) so that this never happens
    if (pl.st_off > pool_records || (REG && (pl.room0 > REG_ROOM || pl.room1 > REG_ROOM))) {
        if (tid == 0) atomicOr(a.err, ERR_POOL);
        return;
    }

    // ---- the first round of the own lists and tables: in flight while the
    //      neighbour counts and records are gathered
    const int tab_len = max(max(n0, n1), max(pl.nln, pl.ncl));
    uint4 f0 = make_uint4(0u, 0u, 0u, 0u), f1 = f0, fc = f0;
    double fl = 0.0, fd = 0.0;
    if (tid < n0) f0 = recb[(size_t)G.cell0 * cap + tid];
    if (tid < n1) f1 = recb[(size_t)G.cell1 * cap + tid];
    if (tid < pl.nln) fl = a.lntab[tid];
    if (tid < pl.ncl) { fc = core_g[tid]; fd = cdel_g[tid]; }

    // ---- neighbour segments: counts, then a wavefront prefix scan -----------
    int cnt = 0;
    uint32_t seg_cell = 0;
    if (lane < 52) {
        const int j = lane / 26;
        if (j < ncell) {
            seg_cell = j ? neighbour_cell(G.cc1[0], G.cc1[1], G.cc1[2], lane - 26, n)
                         : neighbour_cell(G.cc0[0], G.cc0[1], G.cc0[2], lane, n);
            cnt = (int)cntb[seg_cell];
        }
    }
    int pre_v = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(pre_v, off, 64);
        if (lane >= off) pre_v += v;
    }
    const int nb_total = (int)rdl((uint32_t)pre_v, 51);
    const int nbc0 = (int)rdl((uint32_t)pre_v, 25);

    // ---- neighbours: staged in the rest of the pool, the excess read from memory
    const int st_end = min(nb_total, pool_records - pl.st_off);
    {
        // four chunks per round: their loads are in flight together
        int q = 0;
        for (int g0 = 64 * wid; g0 < st_end; g0 += 4 * nt) {
            uint4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int gu = g0 + u * nt;
                v[u] = make_uint4(0u, 0u, 0u, 0u);
                if (gu < st_end) {
                    uint32_t c;
                    int off;
                    chunk_src(gu, lane, q, pre_v, seg_cell, c, off);
                    if (gu + lane < st_end) v[u] = recb[(size_t)c * cap + off];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int gl = g0 + u * nt + lane;
                if (gl < st_end) {
                    uint4 w = v[u];
                    w.w = charge_bits(w.w, a.ion_coupling);
                    pool[pl.st_off + gl] = w;
                }
            }
        }
    }
    const bool spill = nb_total > st_end;
    if (spill && tid == 0) atomicOr(a.err, INFO_UNSTAGED);

    // ---- own lists, ln table, cores -----------------------------------------
    double* lnt = reinterpret_cast<double*>(pool + pl.ln_off);
    uint4* lcore = pool + pl.core_off;
    double* lcdel = reinterpret_cast<double*>(pool + pl.cdel_off);
    {
        if (!REG && tid < n0) pool[tid] = f0;
        if (!REG && tid < n1) pool[pl.room0 + tid] = f1;
        if (tid < pl.nln) lnt[tid] = fl;
        if (tid < pl.ncl) { lcore[tid] = fc; lcdel[tid] = fd; }
        // further rounds (long lists): a share of every table, all in flight together
        for (int i = tid + nt; i < tab_len; i += nt) {
            uint4 r0 = make_uint4(0u, 0u, 0u, 0u), r1 = r0, cx = r0;
            double l = 0.0, dl = 0.0;
            if (i < n0) r0 = recb[(size_t)G.cell0 * cap + i];
            if (i < n1) r1 = recb[(size_t)G.cell1 * cap + i];
            if (i < pl.nln) l = a.lntab[i];
            if (i < pl.ncl) { cx = core_g[i]; dl = cdel_g[i]; }
            if (!REG && i < n0) pool[i] = r0;
            if (!REG && i < n1) pool[pl.room0 + i] = r1;
            if (i < pl.nln) lnt[i] = l;
            if (i < pl.ncl) { lcore[i] = cx; lcdel[i] = dl; }
        }
    }
    if (wpd > 1) __syncthreads(); else wave_sync();
    // a light domain's lists: lane i holds record i of each member (lanes past
    // the count hold stale or zero records and are never read as members)
    uint4 L0 = f0, L1 = f1;
    double D0 = 0.0, D1 = 0.0;

    // ---- learned proposal: site probabilities of the lists, class weights ------
    double* aux = reinterpret_cast<double*>(pool + pl.aux_off);
    ClassW cw{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    // with register lists the p_i sit beside the records and the aux slots hold
    // the eight class weights instead, in the order of ClassW: index 2 c + m
    // for class c (0 neutral acids, 1 ionized acids, 2 neutral bases, 3
    // ionized bases; the sites move c eligible for) and member m
    double* const cwl = aux;
    constexpr bool learned = LEARNED;
    if (learned && REG) {
        const double* phat = R.phat;
        const int k0 = rec_kind(L0.w), k1 = rec_kind(L1.w);
        if (lane < n0 && (k0 == (int)KIND_ACID || k0 == (int)KIND_BASE)) D0 = phat[L0.w >> 8];
        if (lane < n1 && (k1 == (int)KIND_ACID || k1 == (int)KIND_BASE)) D1 = phat[L1.w >> 8];
        double w0, w1, w2, w3, w4, w5, w6, w7;
        class_sums_reg(L0.w, D0, n0, lane, w0, w2, w4, w6);
        class_sums_reg(L1.w, D1, n1, lane, w1, w3, w5, w7);
        if (lane < 8)
            cwl[lane] = lane == 0 ? w0 : lane == 1 ? w1 : lane == 2 ? w2 : lane == 3 ? w3
                      : lane == 4 ? w4 : lane == 5 ? w5 : lane == 6 ? w6 : w7;
        wave_sync();
    } else if (learned) {
        const double* phat = R.phat;
        for (int i = tid; i < n0 + n1; i += nt) {
            const int slot = i < n0 ? i : pl.room0 + (i - n0);
            const uint32_t m = pool[slot].w;
            const int kd = rec_kind(m);
            aux[slot] = (kd == (int)KIND_ACID || kd == (int)KIND_BASE) ? phat[m >> 8] : 0.0;
        }
        if (wpd > 1) __syncthreads(); else wave_sync();
        class_sums(pool, aux, 0, n0, lane, cw.a0_0, cw.ac_0, cw.b0_0, cw.bc_0);
        class_sums(pool, aux, pl.room0, n1, lane, cw.a0_1, cw.ac_1, cw.b0_1, cw.bc_1);
    }

    // ---- counts per member ----------------------------------------------------
    MemberCounts c0 = REG ? count_reg(L0.w, n0, lane) : count_member(pool, 0, n0, lane);
    MemberCounts c1 = REG ? count_reg(L1.w, n1, lane) : count_member(pool, pl.room0, n1, lane);
    const int nsites = c0.a0 + c0.ac + c0.b0 + c0.bc + c1.a0 + c1.ac + c1.b0 + c1.bc;
    // trials of this domain: the state-independent schedule, reaction trials
    // first, then the ion relocation trials
    const int ntr_react = rfl(a.trials * ncell + (nsites * a.site_trials + 15) / 16);
    const int ntr = ntr_react + (RELOC ? a.ion_trials * ncell : 0);
    int react0 = 2, react1 = 2, nreact = 1;
    {
        const bool ha = c0.a0 + c0.ac + c1.a0 + c1.ac > 0, hb = c0.b0 + c0.bc + c1.b0 + c1.bc > 0;
        if (ha && hb) { react0 = 0; react1 = 1; nreact = 3; }
        else if (ha) { react0 = 0; nreact = 2; }
        else if (hb) { react0 = 1; nreact = 2; }
    }

    // insertion regions and volume terms of the members (tables built on the host)
    const uint32_t* bnd = R.bnd;
    const double lnk = ncell == 2 ? a.ln2 : 0.0;
    uint32_t ib0[3], iw0[3], ib1[3], iw1[3];
#pragma unroll
    for (int dd = 0; dd < 3; ++dd) {
        const uint32_t oo = R.tab->o[dd];
        const uint32_t l0 = bnd[G.cc0[dd]], h0 = bnd[G.cc0[dd] + 1];
        const uint32_t l1 = bnd[G.cc1[dd]], h1 = bnd[G.cc1[dd] + 1];
        ib0[dd] = oo + l0; iw0[dd] = h0 - l0;
        ib1[dd] = oo + l1; iw1[dd] = h1 - l1;
    }
    const double lnZm0 = (R.lnZ0 + lnk) + ((R.lnW[G.cc0[0]] + R.lnW[G.cc0[1]]) + R.lnW[G.cc0[2]]);
    const double lnZm1 = (R.lnZ0 + lnk) + ((R.lnW[G.cc1[0]] + R.lnW[G.cc1[1]]) + R.lnW[G.cc1[2]]);

    PairParams P;
    P.scale_f = (float)R.scale;
    P.scale_d = R.scale;
    P.sc2_d = R.scale * R.scale;
    P.sc2_f = (float)P.sc2_d;
    P.kl_d = -R.kappa * 1.4426950408889634074; // log2(e)
    P.kl_f = (float)P.kl_d;
    P.R2 = R.R2;
    P.rc2_f = (float)((double)R.R2 * R.scale * R.scale);
    P.band_f = P.rc2_f * 1.2e-5f;
    P.rc2_lo = (double)R.R2 * R.scale * R.scale * (1.0 - 1e-5);
    P.rc2_hi = (double)R.R2 * R.scale * R.scale * (1.0 + 1e-5);
    P.lB = a.lB;
    P.kappa = R.kappa;
    P.eps = a.eps;
    P.ion_coupling = a.ion_coupling;
    const bool ev_on = a.eps > 0.0 && a.ion_coupling;
    const double lnKA = R.lnKA, lnKB = R.lnKB, lnKion = R.lnKion;

    // attempts and accepts per move, three 21-bit fields per word (moves 0-2, 3-5)
    uint64_t attL = 0, attH = 0, acpL = 0, acpH = 0;
    int rel_att = 0, rel_acc = 0; // ion relocations
    int dA = 0, dB = 0, dXp = 0, dXm = 0; // changes of nA-, nB+, nX+, nX-
    double dE = 0.0;
    uint32_t ph0 = 0, ph1 = 0, ph2 = 0, ph3 = 0;
    int nred = 0;

    // ---- an empty light domain: until its first accepted insertion no trial
    //      changes anything, so ten consecutive trials are evaluated side by
    //      side against the same state (six lanes each, lane 6i + b holding
    //      Philox block b of trial i as in the loop below) and taken in order
    //      up to and including the first accepted one
    int t_first = 0;
    if (FAST && REG && n0 + n1 == 0 && nreact == 1 && !spill) {
        const int grp = lane / 6, sub = lane % 6; // lanes 60-63 idle
        const bool lead = sub == 0 && grp < 10;
        const double lnp_counts = -lnt[1] - lnt[1] + lnKion;
        bool done = false;
        for (int t0 = 0; t0 < ntr && !done; t0 += 10) {
            const int t = t0 + grp;
            const bool live = grp < 10 && t < ntr;
            uint32_t w4[4];
            philox4x32_10((uint32_t)s, G.cell0, (uint32_t)(t0 + lane / 6) * 8u + (uint32_t)(lane % 6), TAG_TRIAL,
                          key0, key1, w4);
            const auto wd = [&](int wi) -> uint32_t {
                const int c = wi & 3;
                const uint32_t v = c == 0 ? w4[0] : (c == 1 ? w4[1] : (c == 2 ? w4[2] : w4[3]));
                return (uint32_t)__shfl((int)v, 6 * grp + (wi >> 2), 64);
            };
            // the salt reaction alone: forward (move 4) or reverse (5, nothing to delete)
            const int move = RELOC && t >= ntr_react ? 6 : 4 + (int)(pick32(wd(0), 2u) & 1u);
            const double u = unit53(wd(16), wd(17));
            const bool ins = live && move == 4;
            Chg A, B;
            const int jA = ncell == 1 ? 0 : (int)pick32(wd(18), (uint32_t)ncell);
            const int jB = ncell == 1 ? 0 : (int)pick32(wd(19), (uint32_t)ncell);
            A.member = jA; A.own = -1; A.ion = 1; A.q_old = 0; A.q_new = 1; A.pres_old = 0; A.pres_new = 1;
            A.dq = a.ion_coupling ? 1 : 0; A.dw = ev_on ? 1 : 0;
            A.x = (jA ? ib1[0] : ib0[0]) + pick64(wd(4), wd(5), jA ? iw1[0] : iw0[0]);
            A.y = (jA ? ib1[1] : ib0[1]) + pick64(wd(6), wd(7), jA ? iw1[1] : iw0[1]);
            A.z = (jA ? ib1[2] : ib0[2]) + pick64(wd(8), wd(9), jA ? iw1[2] : iw0[2]);
            B.member = jB; B.own = -1; B.ion = 1; B.q_old = 0; B.q_new = -1; B.pres_old = 0; B.pres_new = 1;
            B.dq = a.ion_coupling ? -1 : 0; B.dw = ev_on ? 1 : 0;
            B.x = (jB ? ib1[0] : ib0[0]) + pick64(wd(10), wd(11), jB ? iw1[0] : iw0[0]);
            B.y = (jB ? ib1[1] : ib0[1]) + pick64(wd(12), wd(13), jB ? iw1[1] : iw0[1]);
            B.z = (jB ? ib1[2] : ib0[2]) + pick64(wd(14), wd(15), jB ? iw1[2] : iw0[2]);
            const double lnvol = (jB ? lnZm1 : lnZm0) + (jA ? lnZm1 : lnZm0);

            // energy change: the group's six lanes share the member's staged
            // neighbours (the domain's own lists are empty)
            double aqA = 0.0, aqB = 0.0, aw = 0.0;
            int ov = 0;
            float gap = 3.0e38f;
            for (int j = 0; j < ncell; ++j) {
                const int lo = j ? nbc0 : 0, hi = j ? nb_total : nbc0;
                for (int g = lo + sub; g < hi; g += 6) {
                    const uint4 rc = pool[pl.st_off + g];
                    if (ins && jA == j) pair_acc<Real>(rc, rc.w, true, A, P, aqA, aw, ov, gap);
                    if (ins && jB == j) pair_acc<Real>(rc, rc.w, true, B, P, aqB, aw, ov, gap);
                }
            }
            if (__ballot(gap <= P.band_f)) {
                for (int j = 0; j < ncell; ++j) {
                    const int lo = j ? nbc0 : 0, hi = j ? nb_total : nbc0;
                    for (int g = lo + sub; g < hi; g += 6) {
                        const uint4 rc = pool[pl.st_off + g];
                        if (ins && jA == j) pair_band<Real>(rc, rc.w, true, A, P, aqA);
                        if (ins && jB == j) pair_band<Real>(rc, rc.w, true, B, P, aqB);
                    }
                }
            }
            double acc = P.lB * ((double)A.dq * aqA + (double)B.dq * aqB) + aw;
            if (ins && ev_on && ncores) {
                for (int k = sub; k < (int)ncores; k += 6) {
                    const uint4 cx = pl.ncl ? lcore[k] : core_g[k];
                    const double dl = pl.ncl ? lcdel[k] : cdel_g[k];
                    acc += wca_core<Real>(A, cx, dl, P, ov);
                    acc += wca_core<Real>(B, cx, dl, P, ov);
                }
            }
            if (ins && sub == 0) acc += changed_pair<Real>(A, B, P, ev_on, ov);
            // the group's sums, its six lanes added in order
            double dU = 0.0;
            int gov = 0;
            for (int q = 0; q < 6; ++q) {
                dU += __shfl(acc, 6 * grp + q, 64);
                gov |= __shfl(ov, 6 * grp + q, 64);
            }
            if (gov) dU = __longlong_as_double(0x7FF0000000000000ll);
            const double lnp = lnp_counts + lnvol - dU;
            const bool cap_fail = ins && ((jA == 0) + (jB == 0) > (int)cap || (jA == 1) + (jB == 1) > (int)cap);
            const bool accepted = ins && !cap_fail && metropolis(u, lnp);
            // the first accepted trial of the ten; the trials up to it are final
            const uint64_t accm = __ballot(lead && live && accepted);
            const int first = accm ? (int)(__builtin_ctzll(accm) / 6) : 10;
            const bool taken = lead && live && grp <= first;
            attH += (uint64_t)__popcll(__ballot(taken && move == 4)) << 21;
            attH += (uint64_t)__popcll(__ballot(taken && move == 5)) << 42;
            rel_att += __popcll(__ballot(taken && move == 6));
            if (taken && cap_fail) atomicOr(a.err, ERR_INSERT_CAPACITY);
            if (taken && a.log) {
                const unsigned long long li = atomicAdd(a.log_n, 1ull);
                if (li < a.log_cap) {
                    TrialRec& L = a.log[li];
                    L.sweep = (int64_t)s; L.cell = G.cell0; L.trial = t; L.replica = (int32_t)r;
                    L.move = move; L.status = move == 4 ? (accepted ? 1 : 0) : 2;
                    L.dU = move == 4 ? dU : __longlong_as_double(0x7FF8000000000000ll);
                    L.lnp = move == 4 ? lnp : L.dU;
                    L.u = u;
                }
            }
            if (accm) {
                // commit the accepted insertion: cation, then anion, appended
                const int src = 6 * first;
                const int ja = (int)rdl((uint32_t)jA, src), jb = (int)rdl((uint32_t)jB, src);
                const uint32_t ax = rdl(A.x, src), ay = rdl(A.y, src), az = rdl(A.z, src);
                const uint32_t bx = rdl(B.x, src), by = rdl(B.y, src), bz = rdl(B.z, src);
                const long long ub = __double_as_longlong(dU);
                const double dUf =
                    __longlong_as_double((long long)(((uint64_t)rdl((uint32_t)((uint64_t)ub >> 32), src) << 32) |
                                                     (uint64_t)rdl((uint32_t)ub, src)));
                {
                    // the lists were empty: cation and anion in slots 0 and 0, or 0 and 1
                    const uint4 ra = make_uint4(ax, ay, az, make_meta(KIND_XPOS, 1u, NO_SITE));
                    const uint4 rb = make_uint4(bx, by, bz, make_meta(KIND_XNEG, 1u, NO_SITE));
                    if (ja) reg_append(L1, D1, 0, ra, lane); else reg_append(L0, D0, 0, ra, lane);
                    const int sb = ja == jb ? 1 : 0;
                    if (jb) reg_append(L1, D1, sb, rb, lane); else reg_append(L0, D0, sb, rb, lane);
                }
                acpH += 1ull << 21;
                dE += dUf;
                MemberCounts& cma = ja ? c1 : c0;
                MemberCounts& cmb = jb ? c1 : c0;
                ++cma.xp;
                ++cmb.xn;
                dXp += 1;
                dXm += 1;
                n0 += (ja == 0) + (jb == 0);
                n1 += (ja == 1) + (jb == 1);
                t_first = t0 + first + 1;
                done = true;
            } else {
                t_first = min(t0 + 10, ntr);
            }
            wave_sync();
        }
    }

    for (int t = t_first; t < ntr; ++t) {
        // the loop-carried state is uniform: keep it in scalar registers
        n0 = rfl(n0);
        n1 = rfl(n1);
        c0 = rfl_counts(c0);
        c1 = rfl_counts(c1);
        nred = rfl(nred);
        // Philox words, ten trials at a time: lane 6i + b holds block b of
        // trial i of the batch (blocks 0-4 every trial, 5 the learned pick)
        const int tl = t % 10;
        if (tl == 0 || t == t_first) {
            uint32_t w[4];
            philox4x32_10((uint32_t)s, G.cell0, (uint32_t)(t - tl + lane / 6) * 8u + (uint32_t)(lane % 6),
                          TAG_TRIAL, key0, key1, w);
            ph0 = w[0]; ph1 = w[1]; ph2 = w[2]; ph3 = w[3];
        }
        // words 0-3 and 16-19 serve every trial; the insertion coordinates
        // (words 4-15) are read where an insertion needs them
        uint32_t W[20];
#pragma unroll
        for (int b = 0; b < 5; b += 4) {
            const int src = 6 * tl + b;
            W[4 * b + 0] = rdl(ph0, src);
            W[4 * b + 1] = rdl(ph1, src);
            W[4 * b + 2] = rdl(ph2, src);
            W[4 * b + 3] = rdl(ph3, src);
        }
        const auto word = [&](int w) -> uint32_t {
            const int c = w & 3;
            return rdl(c == 0 ? ph0 : (c == 1 ? ph1 : (c == 2 ? ph2 : ph3)), 6 * tl + (w >> 2));
        };

        const uint32_t kk = pick32(W[0], (uint32_t)(2 * nreact));
        const int rsel = (int)(kk >> 1);
        const int reaction = rsel == 0 ? react0 : (rsel == 1 ? react1 : 2);
        const int move = rfl(RELOC && t >= ntr_react ? 6 : 2 * reaction + (int)(kk & 1u));
        const double u = rfld(unit53(W[16], W[17]));
        const int m0a = c0.a0 + c1.a0, mca = c0.ac + c1.ac, m0b = c0.b0 + c1.b0, mcb = c0.bc + c1.bc;
        const int npos = c0.xp + c1.xp, nneg = c0.xn + c1.xn;

        // participants: A is the site (moves 0-3) or the cation (4, 5); B is the
        // ion deleted with it.  Each is the k-th of its class in domain order.
        int a_mem = -1, a_own = -1, b_mem = -1, b_own = -1;
        bool auto_reject = false;
        double lnp_counts = 0.0;
        uint32_t am = 0, av = 0, bm = 0, bv = 0; // classes (mask, value); mask 0: none
        int ak = 0, bk = 0, ac0 = 0, bc0 = 0;   // rank in the domain, count in member 0
        switch (move) {
        case 0:
            auto_reject = m0a == 0;
            am = CLS_MASK_SITE; av = KIND_ACID; ak = (int)pick32(W[1], (uint32_t)m0a); ac0 = c0.a0;
            if (!auto_reject) lnp_counts = lnt[m0a] - lnt[mca + 1] - lnt[npos + 1] + lnKA;
            break;
        case 1:
            auto_reject = mca == 0 || npos == 0;
            am = CLS_MASK_SITE; av = KIND_ACID | 8u; ak = (int)pick32(W[1], (uint32_t)mca); ac0 = c0.ac;
            bm = CLS_MASK_ION; bv = KIND_XPOS; bk = (int)pick32(W[2], (uint32_t)npos); bc0 = c0.xp;
            if (!auto_reject) lnp_counts = lnt[mca] + lnt[npos] - lnt[m0a + 1] - lnKA;
            break;
        case 2:
            auto_reject = m0b == 0;
            am = CLS_MASK_SITE; av = KIND_BASE; ak = (int)pick32(W[1], (uint32_t)m0b); ac0 = c0.b0;
            if (!auto_reject) lnp_counts = lnt[m0b] - lnt[mcb + 1] - lnt[nneg + 1] + lnKB;
            break;
        case 3:
            auto_reject = mcb == 0 || nneg == 0;
            am = CLS_MASK_SITE; av = KIND_BASE | 8u; ak = (int)pick32(W[1], (uint32_t)mcb); ac0 = c0.bc;
            bm = CLS_MASK_ION; bv = KIND_XNEG; bk = (int)pick32(W[3], (uint32_t)nneg); bc0 = c0.xn;
            if (!auto_reject) lnp_counts = lnt[mcb] + lnt[nneg] - lnt[m0b + 1] - lnKB;
            break;
        case 4:
            lnp_counts = -lnt[npos + 1] - lnt[nneg + 1] + lnKion;
            break;
        case 5:
            auto_reject = npos == 0 || nneg == 0;
            am = CLS_MASK_ION; av = KIND_XPOS; ak = (int)pick32(W[2], (uint32_t)npos); ac0 = c0.xp;
            bm = CLS_MASK_ION; bv = KIND_XNEG; bk = (int)pick32(W[3], (uint32_t)nneg); bc0 = c0.xn;
            if (!auto_reject) lnp_counts = lnt[npos] + lnt[nneg] - lnKion;
            break;
        default:
            if (RELOC) {
                // ion relocation: the k-th free ion of the domain, cations first
                auto_reject = npos + nneg == 0;
                const int k = (int)pick32(W[1], (uint32_t)(npos + nneg));
                am = CLS_MASK_ION;
                if (k < npos) { av = KIND_XPOS; ak = k; ac0 = c0.xp; }
                else { av = KIND_XNEG; ak = k - npos; ac0 = c0.xn; }
            }
            break;
        }
        // learned site pick (moves 0-3): uniform with probability eps (word
        // 20), else by weight (words 21, 22)
        bool weighted = false;
        double lp_w = 0.0, lp_W0 = 0.0, lp_W1 = 0.0;
        if (learned && move <= 3 && !auto_reject) {
            const int src = 6 * tl + 5;
            const uint32_t we = rdl(ph0, src), wt0 = rdl(ph1, src), wt1 = rdl(ph2, src);
            weighted = !((double)we * (1.0 / 4294967296.0) < a.learn_eps);
            if (REG) {
                lp_W0 = cwl[2 * move];
                lp_W1 = cwl[2 * move + 1];
            } else {
                lp_W0 = move == 0 ? cw.a0_0 : move == 1 ? cw.ac_0 : move == 2 ? cw.b0_0 : cw.bc_0;
                lp_W1 = move == 0 ? cw.a0_1 : move == 1 ? cw.ac_1 : move == 2 ? cw.b0_1 : cw.bc_1;
            }
            if (weighted) {
                const double target = unit53(wt0, wt1) * (lp_W0 + lp_W1);
                const int mem = (target < lp_W0 && lp_W0 > 0.0) || lp_W1 <= 0.0 ? 0 : 1;
                a_mem = mem;
                a_own = REG ? rfl(reg_kth_weighted(mem ? L1.w : L0.w, mem ? D1 : D0, mem ? n1 : n0, am, av,
                                                   !(move & 1), mem ? target - lp_W0 : target, lane))
                            : rfl(member_kth_weighted(pool, aux, mem ? pl.room0 : 0, mem ? n1 : n0, am, av,
                                                      !(move & 1), mem ? target - lp_W0 : target, lane));
            }
        }
        if (!auto_reject) {
#pragma unroll 1
            for (int pidx = weighted ? 1 : 0; pidx < 2; ++pidx) {
                const uint32_t cm = pidx ? bm : am, cv = pidx ? bv : av;
                if (!cm) continue;
                const int k = pidx ? bk : ak, k0 = pidx ? bc0 : ac0;
                const int mem = k < k0 ? 0 : 1;
                const int own = REG ? rfl(reg_kth(mem ? L1.w : L0.w, mem ? n1 : n0, cm, cv, mem ? k - k0 : k, lane))
                                    : rfl(member_kth(pool, mem ? pl.room0 : 0, mem ? n1 : n0, cm, cv,
                                                     mem ? k - k0 : k, lane));
                if (pidx) { b_mem = mem; b_own = own; } else { a_mem = mem; a_own = own; }
            }
            if (learned && move <= 3) {
                // ln q_rev(i | s') - ln q_fwd(i | s) replaces the count ratio
                const bool fwd = !(move & 1);
                const double p_i = REG ? lane_d(a_mem ? D1 : D0, a_own) : rfld(aux[(a_mem ? pl.room0 : 0) + a_own]);
                const double wi = fwd ? p_i : 1.0 - p_i, wr = 1.0 - wi;
                const int m = move == 0 ? m0a : move == 1 ? mca : move == 2 ? m0b : mcb;
                const int mr = (move == 0 ? mca : move == 1 ? m0a : move == 2 ? mcb : m0b) + 1;
                const double Wr = (REG ? cwl[2 * (move ^ 1)] + cwl[2 * (move ^ 1) + 1]
                                       : move == 0 ? cw.ac_0 + cw.ac_1 : move == 1 ? cw.a0_0 + cw.a0_1
                                       : move == 2 ? cw.bc_0 + cw.bc_1 : cw.b0_0 + cw.b0_1) + wr;
                const double eps = a.learn_eps;
                const double lnq = log(eps / mr + (1.0 - eps) * wr / Wr) - log(eps / m + (1.0 - eps) * wi / (lp_W0 + lp_W1));
                lp_w = p_i;
                switch (move) {
                case 0: lnp_counts = lnq - lnt[npos + 1] + lnKA; break;
                case 1: lnp_counts = lnq + lnt[npos] - lnKA; break;
                case 2: lnp_counts = lnq - lnt[nneg + 1] + lnKB; break;
                default: lnp_counts = lnq + lnt[nneg] - lnKB; break;
                }
            }
        }
        const uint64_t mv_one = 1ull << (21 * (move % 3));
        if (move < 3) attL += mv_one; else if (!RELOC || move < 6) attH += mv_one; else ++rel_att;
        if (auto_reject) {
            if (tid == 0 && a.log) {
                const unsigned long long li = atomicAdd(a.log_n, 1ull);
                if (li < a.log_cap) {
                    TrialRec& L = a.log[li];
                    L.sweep = (int64_t)s; L.cell = G.cell0; L.trial = t; L.replica = (int32_t)r;
                    L.move = move; L.status = 2;
                    L.dU = __longlong_as_double(0x7FF8000000000000ll); L.lnp = L.dU; L.u = u;
                }
            }
            continue;
        }

        // ---- the two changed particles (uniform) ------------------------------
        Chg A, B;
        double lnvol = 0.0;
        const bool insertion = move == 0 || move == 2 || move == 4;
        if (RELOC && move == 6) {
            // ion relocation: A is the ion leaving its place, B the same ion at
            // a point drawn like an insertion of its sign
            const int q = av == KIND_XPOS ? 1 : -1;
            const uint4 rc = REG ? lane_rec(a_mem ? L1 : L0, a_own) : pool[pl.base(a_mem) + a_own];
            A.member = a_mem; A.own = a_own;
            A.x = rflu(rc.x); A.y = rflu(rc.y); A.z = rflu(rc.z);
            A.ion = 1; A.q_old = q; A.q_new = 0; A.pres_old = 1; A.pres_new = 0;
            A.dq = a.ion_coupling ? -q : 0;
            A.dw = ev_on ? -1 : 0;
            lnvol -= a_mem ? lnZm1 : lnZm0;
            const uint32_t wc = q > 0 ? W[18] : W[19];
            const int wo = q > 0 ? 4 : 10;
            const int j = ncell == 1 ? 0 : (int)pick32(wc, (uint32_t)ncell);
            B.member = j; B.own = -1;
            B.x = (j ? ib1[0] : ib0[0]) + pick64(word(wo + 0), word(wo + 1), j ? iw1[0] : iw0[0]);
            B.y = (j ? ib1[1] : ib0[1]) + pick64(word(wo + 2), word(wo + 3), j ? iw1[1] : iw0[1]);
            B.z = (j ? ib1[2] : ib0[2]) + pick64(word(wo + 4), word(wo + 5), j ? iw1[2] : iw0[2]);
            B.ion = 1; B.q_old = 0; B.q_new = q; B.pres_old = 0; B.pres_new = 1;
            B.dq = a.ion_coupling ? q : 0;
            B.dw = ev_on ? 1 : 0;
            lnvol += j ? lnZm1 : lnZm0;
        }
        if (move <= 3) {
            // A: the site flips
            const uint4 rc = REG ? lane_rec(a_mem ? L1 : L0, a_own) : pool[pl.base(a_mem) + a_own];
            A.member = a_mem; A.own = a_own;
            A.x = rflu(rc.x); A.y = rflu(rc.y); A.z = rflu(rc.z);
            const uint32_t mw = rflu(rc.w);
            const int chg = rec_charged(mw);
            const int sgn = rec_kind(mw) == (int)KIND_ACID ? -1 : 1;
            A.q_old = sgn * chg; A.q_new = sgn * (1 - chg);
            A.dq = A.q_new - A.q_old; A.dw = 0; A.ion = 0; A.pres_old = 1; A.pres_new = 1;
        }
        if (!RELOC || move < 6) {
            // B (and A for salt moves): ions in or out
            const int qB = (move <= 1) ? 1 : -1; // cation for acid moves, anion otherwise
            B.ion = 1;
            B.q_old = insertion ? 0 : qB;
            B.q_new = insertion ? qB : 0;
            B.pres_old = insertion ? 0 : 1;
            B.pres_new = insertion ? 1 : 0;
            B.dq = a.ion_coupling ? B.q_new - B.q_old : 0;
            B.dw = ev_on ? (insertion ? 1 : -1) : 0;
            if (insertion) {
                const uint32_t wc = qB > 0 ? W[18] : W[19];
                const int wo = qB > 0 ? 4 : 10;
                const int j = ncell == 1 ? 0 : (int)pick32(wc, (uint32_t)ncell);
                B.member = j;
                B.own = -1;
                B.x = (j ? ib1[0] : ib0[0]) + pick64(word(wo + 0), word(wo + 1), j ? iw1[0] : iw0[0]);
                B.y = (j ? ib1[1] : ib0[1]) + pick64(word(wo + 2), word(wo + 3), j ? iw1[1] : iw0[1]);
                B.z = (j ? ib1[2] : ib0[2]) + pick64(word(wo + 4), word(wo + 5), j ? iw1[2] : iw0[2]);
                lnvol += j ? lnZm1 : lnZm0;
            } else {
                const uint4 rc = REG ? lane_rec(b_mem ? L1 : L0, b_own) : pool[pl.base(b_mem) + b_own];
                B.member = b_mem; B.own = b_own;
                B.x = rflu(rc.x); B.y = rflu(rc.y); B.z = rflu(rc.z);
                lnvol -= b_mem ? lnZm1 : lnZm0;
            }
        }
        if (move == 4 || move == 5) {
            A.ion = 1;
            A.q_old = insertion ? 0 : 1;
            A.q_new = insertion ? 1 : 0;
            A.pres_old = insertion ? 0 : 1;
            A.pres_new = insertion ? 1 : 0;
            A.dq = a.ion_coupling ? A.q_new - A.q_old : 0;
            A.dw = ev_on ? (insertion ? 1 : -1) : 0;
            if (insertion) {
                const int j = ncell == 1 ? 0 : (int)pick32(W[18], (uint32_t)ncell);
                A.member = j;
                A.own = -1;
                A.x = (j ? ib1[0] : ib0[0]) + pick64(word(4), word(5), j ? iw1[0] : iw0[0]);
                A.y = (j ? ib1[1] : ib0[1]) + pick64(word(6), word(7), j ? iw1[1] : iw0[1]);
                A.z = (j ? ib1[2] : ib0[2]) + pick64(word(8), word(9), j ? iw1[2] : iw0[2]);
                lnvol += j ? lnZm1 : lnZm0;
            } else {
                const uint4 rc = REG ? lane_rec(a_mem ? L1 : L0, a_own) : pool[pl.base(a_mem) + a_own];
                A.member = a_mem; A.own = a_own;
                A.x = rflu(rc.x); A.y = rflu(rc.y); A.z = rflu(rc.z);
                lnvol -= a_mem ? lnZm1 : lnZm0;
            }
        }
        uniform_chg(A);
        uniform_chg(B);
        lnvol = rfld(lnvol);
        lnp_counts = rfld(lnp_counts);
        // per-member growth check against the cell capacity
        const int gA = A.pres_new - A.pres_old, gB = B.pres_new - B.pres_old;
        const int grow0 = (A.member == 0 ? gA : 0) + (B.member == 0 ? gB : 0);
        const int grow1 = (A.member == 1 ? gA : 0) + (B.member == 1 ? gB : 0);
        const bool cap_fail = n0 + grow0 > (int)cap || n1 + grow1 > (int)cap;

        // ---- energy change: every lane sums a share of the records -----------
        // member j's own list (changing: read from the pool), its staged
        // neighbour slots, and any neighbours left in memory
        double aqA = 0.0, aqB = 0.0, aw = 0.0;
        int ov = 0;
        float gap = 3.0e38f;
#pragma unroll 1
        for (int j = 0; j < ncell; ++j) {
            const bool inA = A.member == j, inB = B.member == j;
            if (!inA && !inB) continue;
            const int bs = pl.base(j), nn = j ? n1 : n0;
            const int skA = inA ? A.own : -1, skB = inB ? B.own : -1;
            if (REG) {
                if (nn > 0) {
                    const bool v = lane < nn && lane != skA && lane != skB;
                    const uint4 rc = j ? L1 : L0;
                    const uint32_t code = charge_bits(rc.w, P.ion_coupling);
                    if (inA) pair_acc<Real>(rc, code, v, A, P, aqA, aw, ov, gap);
                    if (inB) pair_acc<Real>(rc, code, v, B, P, aqB, aw, ov, gap);
                }
            } else {
                for (int g0 = 0; g0 < nn; g0 += nt) {
                    const int g = g0 + tid;
                    const bool v = g < nn && g != skA && g != skB;
                    const uint4 rc = pool[bs + min(g, nn - 1)];
                    const uint32_t code = charge_bits(rc.w, P.ion_coupling);
                    if (inA) pair_acc<Real>(rc, code, v, A, P, aqA, aw, ov, gap);
                    if (inB) pair_acc<Real>(rc, code, v, B, P, aqB, aw, ov, gap);
                }
            }
            const int lo = j ? nbc0 : 0, hi = j ? nb_total : nbc0;
            const int s1 = min(hi, st_end);
#pragma unroll 2
            for (int g0 = lo; g0 < s1; g0 += nt) {
                const int g = g0 + tid;
                const bool v = g < s1;
                const uint4 rc = pool[pl.st_off + min(g, s1 - 1)];
                if (inA) pair_acc<Real>(rc, rc.w, v, A, P, aqA, aw, ov, gap);
                if (inB) pair_acc<Real>(rc, rc.w, v, B, P, aqB, aw, ov, gap);
            }
            if (hi > st_end) {
                int q = 0;
                const int m0 = max(lo, st_end);
                for (int g0 = m0 + 64 * wid; g0 < hi; g0 += nt) {
                    uint32_t c;
                    int off;
                    chunk_src(g0, lane, q, pre_v, seg_cell, c, off);
                    const bool v = g0 + lane < hi;
                    const uint4 rc = v ? recb[(size_t)c * cap + off] : make_uint4(0u, 0u, 0u, 0u);
                    const uint32_t code = charge_bits(rc.w, P.ion_coupling);
                    if (inA) pair_acc<Real>(rc, code, v, A, P, aqA, aw, ov, gap);
                    if (inB) pair_acc<Real>(rc, code, v, B, P, aqB, aw, ov, gap);
                }
            }
        }
        if (__ballot(gap <= P.band_f)) {
            // records within 1e-5 of the cutoff (rare): the exact integer test
#pragma unroll 1
            for (int j = 0; j < ncell; ++j) {
                const bool inA = A.member == j, inB = B.member == j;
                if (!inA && !inB) continue;
                const int bs = pl.base(j), nn = j ? n1 : n0;
                const int skA = inA ? A.own : -1, skB = inB ? B.own : -1;
                if (REG) {
                    if (nn > 0) {
                        const bool v = lane < nn && lane != skA && lane != skB;
                        const uint4 rc = j ? L1 : L0;
                        const uint32_t code = charge_bits(rc.w, P.ion_coupling);
                        if (inA) pair_band<Real>(rc, code, v, A, P, aqA);
                        if (inB) pair_band<Real>(rc, code, v, B, P, aqB);
                    }
                } else {
                    for (int g0 = 0; g0 < nn; g0 += nt) {
                        const int g = g0 + tid;
                        const bool v = g < nn && g != skA && g != skB;
                        const uint4 rc = pool[bs + min(g, nn - 1)];
                        const uint32_t code = charge_bits(rc.w, P.ion_coupling);
                        if (inA) pair_band<Real>(rc, code, v, A, P, aqA);
                        if (inB) pair_band<Real>(rc, code, v, B, P, aqB);
                    }
                }
                const int lo = j ? nbc0 : 0, hi = j ? nb_total : nbc0;
                const int s1 = min(hi, st_end);
                for (int g0 = lo; g0 < s1; g0 += nt) {
                    const int g = g0 + tid;
                    const bool v = g < s1;
                    const uint4 rc = pool[pl.st_off + min(g, s1 - 1)];
                    if (inA) pair_band<Real>(rc, rc.w, v, A, P, aqA);
                    if (inB) pair_band<Real>(rc, rc.w, v, B, P, aqB);
                }
                if (hi > st_end) {
                    int q = 0;
                    const int m0 = max(lo, st_end);
                    for (int g0 = m0 + 64 * wid; g0 < hi; g0 += nt) {
                        uint32_t c;
                        int off;
                        chunk_src(g0, lane, q, pre_v, seg_cell, c, off);
                        const bool v = g0 + lane < hi;
                        const uint4 rc = v ? recb[(size_t)c * cap + off] : make_uint4(0u, 0u, 0u, 0u);
                        const uint32_t code = charge_bits(rc.w, P.ion_coupling);
                        if (inA) pair_band<Real>(rc, code, v, A, P, aqA);
                        if (inB) pair_band<Real>(rc, code, v, B, P, aqB);
                    }
                }
            }
        }
        double acc = P.lB * ((double)A.dq * aqA + (double)B.dq * aqB) + aw;
        if (ev_on && ncores && (A.dw != 0 || B.dw != 0)) {
            for (int k = tid; k < (int)ncores; k += nt) {
                const uint4 cx = pl.ncl ? lcore[k] : core_g[k];
                const double dl = pl.ncl ? lcdel[k] : cdel_g[k];
                if (A.dw != 0) acc += wca_core<Real>(A, cx, dl, P, ov);
                if (B.dw != 0) acc += wca_core<Real>(B, cx, dl, P, ov);
            }
        }
        if (tid == 0) acc += changed_pair<Real>(A, B, P, ev_on, ov);
        double dU = wave_sum_dpp(acc);
        int any_ov = __ballot(ov) != 0ull;
        if (wpd > 1) {
            // alternate buffers by reduction: between two writes of one buffer
            // every wavefront has passed the other reduction's barrier, so it
            // has read the first
            const int par = nred & 1;
            ++nred;
            if (lane == 0) { red[par][wid] = dU; ovf[par][wid] = any_ov; }
            __syncthreads();
            dU = ((red[par][0] + red[par][1]) + red[par][2]) + red[par][3];
            any_ov = ovf[par][0] | ovf[par][1] | ovf[par][2] | ovf[par][3];
        }
        // every lane holds the same sums: make that explicit, so that the
        // decision and the loop stay scalar
        dU = rfld(dU);
        if (rfl(any_ov)) dU = __longlong_as_double(0x7FF0000000000000ll);
        const double lnp = lnp_counts + lnvol - dU;
        const bool accept = rfl(!cap_fail && metropolis(u, lnp)) != 0;
        if (tid == 0) {
            if (cap_fail) atomicOr(a.err, ERR_INSERT_CAPACITY);
            if (a.log) {
                const unsigned long long li = atomicAdd(a.log_n, 1ull);
                if (li < a.log_cap) {
                    TrialRec& L = a.log[li];
                    L.sweep = (int64_t)s; L.cell = G.cell0; L.trial = t; L.replica = (int32_t)r;
                    L.move = move; L.status = accept ? 1 : 0;
                    L.dU = dU; L.lnp = lnp; L.u = u;
                }
            }
        }
        if (!accept) continue;

        // ---- commit: flip; deletions (higher index first within one cell);
        //      insertions appended, cation before anion -----------------------
        if (move < 3) acpL += mv_one; else if (!RELOC || move < 6) acpH += mv_one; else ++rel_acc;
        dE += dU;
        if (REG) {
            // the same edits of the register lists, every lane taking part
            if (move <= 3 && lane == A.own) {
                if (A.member) L1.w ^= 8u;
                else L0.w ^= 8u;
            }
            int l0 = n0, l1 = n1;
            const auto rm = [&](int mem, int idx) {
                if (mem) { reg_remove(L1, D1, idx, l1, lane, learned); --l1; }
                else { reg_remove(L0, D0, idx, l0, lane, learned); --l0; }
            };
            const auto ap = [&](int mem, uint4 v) {
                if (mem) { reg_append(L1, D1, l1, v, lane); ++l1; }
                else { reg_append(L0, D0, l0, v, lane); ++l0; }
            };
            const uint4 recB = make_uint4(B.x, B.y, B.z, make_meta(B.q_new > 0 ? KIND_XPOS : KIND_XNEG, 1u, NO_SITE));
            if (RELOC && move == 6) {
                rm(A.member, A.own);
                ap(B.member, recB);
            } else if (!insertion) {
                int dm0 = B.member, di0 = B.own, dm1 = -1, di1 = -1;
                if (move == 5) {
                    dm0 = A.member; di0 = A.own; dm1 = B.member; di1 = B.own;
                    if (dm0 == dm1 && di1 > di0) {
                        const int t0 = di0; di0 = di1; di1 = t0;
                    }
                }
                rm(dm0, di0);
                if (dm1 >= 0) rm(dm1, di1);
            } else {
                if (move == 4) ap(A.member, make_uint4(A.x, A.y, A.z, make_meta(KIND_XPOS, 1u, NO_SITE)));
                ap(B.member, recB);
            }
        } else if (tid == 0) {
            if (move <= 3) pool[pl.base(A.member) + A.own].w ^= 8u;
            int l0 = n0, l1 = n1;
            if (RELOC && move == 6) {
                // the ion leaves its slot like a deletion, then is appended
                int& cn = A.member ? l1 : l0;
                const int bs = pl.base(A.member);
                pool[bs + A.own] = pool[bs + cn - 1];
                if (learned) aux[bs + A.own] = aux[bs + cn - 1];
                --cn;
                int& cm = B.member ? l1 : l0;
                pool[pl.base(B.member) + cm] =
                    make_uint4(B.x, B.y, B.z, make_meta(B.q_new > 0 ? KIND_XPOS : KIND_XNEG, 1u, NO_SITE));
                if (learned) aux[pl.base(B.member) + cm] = 0.0;
                ++cm;
            } else if (!insertion) {
                // deleted: B always; A too for the salt move
                int dm0 = B.member, di0 = B.own, dm1 = -1, di1 = -1;
                if (move == 5) {
                    // the cation (A) first unless the anion sits higher in the same cell
                    dm0 = A.member; di0 = A.own; dm1 = B.member; di1 = B.own;
                    if (dm0 == dm1 && di1 > di0) {
                        const int t0 = di0; di0 = di1; di1 = t0;
                    }
                }
                {
                    int& cn = dm0 ? l1 : l0;
                    const int bs = pl.base(dm0);
                    pool[bs + di0] = pool[bs + cn - 1];
                    if (learned) aux[bs + di0] = aux[bs + cn - 1];
                    --cn;
                }
                if (dm1 >= 0) {
                    int& cn = dm1 ? l1 : l0;
                    const int bs = pl.base(dm1);
                    pool[bs + di1] = pool[bs + cn - 1];
                    if (learned) aux[bs + di1] = aux[bs + cn - 1];
                    --cn;
                }
            } else {
                if (move == 4) {
                    int& cn = A.member ? l1 : l0;
                    pool[pl.base(A.member) + cn] = make_uint4(A.x, A.y, A.z, make_meta(KIND_XPOS, 1u, NO_SITE));
                    if (learned) aux[pl.base(A.member) + cn] = 0.0;
                    ++cn;
                }
                int& cn = B.member ? l1 : l0;
                pool[pl.base(B.member) + cn] =
                    make_uint4(B.x, B.y, B.z, make_meta(B.q_new > 0 ? KIND_XPOS : KIND_XNEG, 1u, NO_SITE));
                if (learned) aux[pl.base(B.member) + cn] = 0.0;
                ++cn;
            }
        }
        // class weights of the learned picks: the flipped site changes class
        if (learned && move <= 3) {
            const double p = lp_w, q = 1.0 - lp_w;
            const bool m1 = A.member != 0;
            if (REG) {
                // every lane makes the same two updates of the same slots
                const int c = 2 * move + (m1 ? 1 : 0), cr = 2 * (move ^ 1) + (m1 ? 1 : 0);
                cwl[c] -= (move & 1) ? q : p;
                cwl[cr] += (move & 1) ? p : q;
            } else switch (move) {
            case 0: if (m1) { cw.a0_1 -= p; cw.ac_1 += q; } else { cw.a0_0 -= p; cw.ac_0 += q; } break;
            case 1: if (m1) { cw.ac_1 -= q; cw.a0_1 += p; } else { cw.ac_0 -= q; cw.a0_0 += p; } break;
            case 2: if (m1) { cw.b0_1 -= p; cw.bc_1 += q; } else { cw.b0_0 -= p; cw.bc_0 += q; } break;
            default: if (m1) { cw.bc_1 -= q; cw.b0_1 += p; } else { cw.bc_0 -= q; cw.b0_0 += p; } break;
            }
        }
        // counts
        if (RELOC && move == 6) {
            const int pos = B.q_new > 0;
            MemberCounts& ca = A.member ? c1 : c0;
            MemberCounts& cb = B.member ? c1 : c0;
            if (pos) { --ca.xp; ++cb.xp; } else { --ca.xn; ++cb.xn; }
        } else {
            apply_counts(c0, move, A.member == 0, B.member == 0);
            apply_counts(c1, move, A.member == 1, B.member == 1);
            const int sg = (move & 1) ? -1 : 1;
            dA += move <= 1 ? sg : 0;
            dB += (move == 2 || move == 3) ? sg : 0;
            dXp += (move <= 1 || move >= 4) ? sg : 0;
            dXm += move >= 2 ? sg : 0;
        }
        n0 += grow0;
        n1 += grow1;
        if (wpd > 1) __syncthreads(); else if (!REG) wave_sync();
    }

    // ---- write the domain's cells back ----------------------------------------
    if (REG) {
        if (lane < n0) recb[(size_t)G.cell0 * cap + lane] = L0;
        if (lane < n1) recb[(size_t)G.cell1 * cap + lane] = L1;
    } else {
        if (wpd > 1) __syncthreads(); else wave_sync();
        for (int i = tid; i < n0; i += nt) recb[(size_t)G.cell0 * cap + i] = pool[i];
        for (int i = tid; i < n1; i += nt) recb[(size_t)G.cell1 * cap + i] = pool[pl.room0 + i];
    }
    if (tid == 0) {
        cntb[G.cell0] = (uint32_t)n0;
        if (ncell == 2) cntb[G.cell1] = (uint32_t)n1;
        if (dE != 0.0) R.e_acc[G.cell0] += dE;
        // the domain's stripe of the replica's counters (k_sweep_end folds them)
        uint32_t* ct = R.ctr + (size_t)(gd % (uint32_t)CTR_STRIPES) * CTR_STRIDE;
        for (int i = 0; i < 6; ++i) {
            const int sh = 21 * (i % 3);
            const uint32_t na = (uint32_t)(((i < 3 ? attL : attH) >> sh) & 0x1FFFFFull);
            const uint32_t nc = (uint32_t)(((i < 3 ? acpL : acpH) >> sh) & 0x1FFFFFull);
            if (na) atomicAdd(&ct[i], na);
            if (nc) atomicAdd(&ct[6 + i], nc);
        }
        if (rel_att) atomicAdd(&ct[12], (uint32_t)rel_att);
        if (rel_acc) atomicAdd(&ct[13], (uint32_t)rel_acc);
        if (dA) atomicAdd(&ct[14], (uint32_t)dA);
        if (dB) atomicAdd(&ct[15], (uint32_t)dB);
        if (dXp) atomicAdd(&ct[16], (uint32_t)dXp);
        if (dXm) atomicAdd(&ct[17], (uint32_t)dXm);
        if (a.trace) {
            const unsigned long long ti = atomicAdd(a.trace_n, 1ull);
            if (ti < a.trace_cap) {
                PhaseTrace& T = a.trace[ti];
                T.t0 = t_start;
                T.t1 = wall_clock64();
                T.sweep = (uint32_t)s; T.domain = gd; T.colour = colour; T.ntr = ntr;
                T.nb = nb_total; T.own = n0 + n1; T.staged = spill ? 0 : 1;
                T.hw = (int32_t)(wpd * 1000 + (int)__smid());
            }
        }
    }
}

extern __shared__ uint4 smem[];

// heavy domains first (one workgroup each), then light ones (four per
// workgroup, one per wavefront); the grid is an upper bound.  The learned
// proposal's code is compiled only into the LEARNED instances, the ion
// relocation trials only into the RELOC ones and the side-by-side trials of
// empty domains only into k_phase_fast (batches with sparse replicas, plain
// proposal), so that the plain kernel keeps its register budget (three
// wavefronts per SIMD).
template <typename Real, bool LEARNED, bool RELOC, bool FAST>
__device__ __forceinline__ void phase_body(const SweepArgs& a)
{
    __shared__ double red[2][4];
    __shared__ int ovf[2][4];
    const int colour = a.colour;
    const uint32_t nh = a.plan_n[plan_idx(colour, PLAN_HEAVY)], nl = a.plan_n[plan_idx(colour, PLAN_LIGHT)];
    const uint32_t b = blockIdx.x;
    const int wave = (int)(threadIdx.x >> 6);
    const bool heavy = b < nh;
    const uint32_t j = heavy ? b : (b - nh) * 4u + (uint32_t)wave;
    if (!heavy && j >= nl) return;
    const int q = heavy ? a.pool : a.pool / 4;
    const size_t slot = (size_t)colour * a.ndom_total + j;
    const uint32_t gd = heavy ? a.plan_heavy[slot] : a.plan_light[slot];
    const uint4 geo = heavy ? a.plan_geo_heavy[slot] : a.plan_geo_light[slot];
    if (heavy) run_domain<Real, LEARNED, RELOC, FAST, 4, false>(a, gd, geo, smem, q, wave, red, ovf);
    else if (geo.x & GEO_REG)
        run_domain<Real, LEARNED, RELOC, FAST, 1, true>(a, gd, geo, smem + (size_t)wave * q, q, 0, red, ovf);
    else run_domain<Real, LEARNED, RELOC, FAST, 1, false>(a, gd, geo, smem + (size_t)wave * q, q, 0, red, ovf);
}

template <typename Real, bool LEARNED, bool RELOC>
__global__ __launch_bounds__(PHASE_THREADS) void k_phase(SweepArgs a)
{
    phase_body<Real, LEARNED, RELOC, false>(a);
}

// The FP32 learned instances are held to three wavefronts per SIMD (a few
// registers spill): a tuned LDS pool of 3072 records allows three workgroups
// per compute unit, and at two wavefronts the suspension's phase takes 30 %
// longer.
template <bool RELOC>
__global__ __launch_bounds__(PHASE_THREADS) __attribute__((amdgpu_waves_per_eu(3))) void k_phase_learned32(SweepArgs a)
{
    phase_body<float, true, RELOC, false>(a);
}

// the FAST instances hold their register use to four wavefronts per SIMD
// (with spills): the batches they serve are bound by how many domains are
// in flight (the chain batch: 4 waves 20 % faster than 3, 5 no better)
template <typename Real, bool RELOC>
__global__ __launch_bounds__(PHASE_THREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_phase_fast(SweepArgs a)
{
    phase_body<Real, false, RELOC, true>(a);
}

// ------------------------------------------------------------------------
// k_sweep_end: counters, series row, group histograms, the next shift
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sweep_end(SweepArgs a)
{
    const uint64_t s = *a.sweep;
    // one wavefront per replica
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t r = blockIdx.x * (blockDim.x / 64u) + (threadIdx.x >> 6);
    if (r >= a.nrep) return;
    const Replica& R = a.reps[r];
    // fold the sweep's counter stripes (lane i holds stripes i, i + 64, ...)
    // into the replica's counters and clear them
    static_assert(CTR_STRIPES % 64 == 0 && CTR_STRIDE >= 20 && CTR_STRIDE % 4 == 0, "whole stripes per lane, in 16-byte pieces");
    {
        constexpr int SPL = CTR_STRIPES / 64;
        // the counters as they stand, read before any stripe is cleared
        uint64_t mv[14];
        int64_t tot[4];
#pragma unroll
        for (int i = 0; i < 14; ++i) mv[i] = R.moves[i];
#pragma unroll
        for (int j = 0; j < 4; ++j) tot[j] = R.totals[j];
        uint32_t v[20]; // counters 0-17 and two unused words, in 16-byte pieces
#pragma unroll
        for (int i = 0; i < 20; ++i) v[i] = 0u;
#pragma unroll
        for (int q = 0; q < SPL; ++q) {
            const uint4* st = reinterpret_cast<const uint4*>(R.ctr + (size_t)(lane + 64u * q) * CTR_STRIDE);
#pragma unroll
            for (int i = 0; i < 5; ++i) {
                const uint4 w = st[i];
                v[4 * i] += w.x; v[4 * i + 1] += w.y; v[4 * i + 2] += w.z; v[4 * i + 3] += w.w;
            }
        }
#pragma unroll
        for (int q = 0; q < SPL; ++q) {
            uint4* st = reinterpret_cast<uint4*>(R.ctr + (size_t)(lane + 64u * q) * CTR_STRIDE);
#pragma unroll
            for (int i = 0; i < 5; ++i) st[i] = make_uint4(0u, 0u, 0u, 0u);
        }
        uint32_t x[18];
#pragma unroll
        for (int i = 0; i < 18; ++i) x[i] = wave_sum_u32(v[i]);
        // the new totals are kept in registers: the series row takes them
        // from there, not from the memory lane 0 writes
#pragma unroll
        for (int j = 0; j < 4; ++j) tot[j] += (int64_t)(int32_t)x[14 + j];
        if (lane == 0) {
#pragma unroll
            for (int i = 0; i < 14; ++i) R.moves[i] = mv[i] + (uint64_t)x[i];
#pragma unroll
            for (int j = 0; j < 4; ++j) R.totals[j] = tot[j];
        }
        if (lane < 4 && R.series_cap > 0) {
            const int64_t row = (int64_t)(s % (uint64_t)R.series_cap);
            R.series[row * 4 + lane] = (int32_t)(lane == 0 ? tot[0] : (lane == 1 ? tot[1] : (lane == 2 ? tot[2] : tot[3])));
        }
    }
    // ionized sites per group at the start of this sweep (counted by the
    // re-binning); the slot is cleared for the sweep after next
    int32_t* gc = R.group_count + (s & 1u) * R.ngroups;
    for (uint32_t g = lane; g < R.ngroups; g += 64u) {
        R.group_hist[R.group_hist_off[g] + gc[g]] += 1;
        gc[g] = 0;
    }
    // the next sweep's shift and this one's, so that its re-binning need not
    // draw them in every wavefront
    if (lane == 0) {
        SweepTab* T = R.tab;
        uint32_t nx[3];
        grid_shift(R.key0, R.key1, s + 1u, a.fixed_grid, nx);
        for (int d = 0; d < 3; ++d) { T->prev[d] = T->o[d]; T->next[d] = nx[d]; }
        T->valid = s + 2u;
    }
}

// the sweep counter, advanced once every replica's end-of-sweep work has read it
__global__ __launch_bounds__(64) void k_sweep_advance(SweepArgs a)
{
    if (threadIdx.x == 0) *a.sweep = *a.sweep + 1u;
}

// ------------------------------------------------------------------------
// k_ungroup: every free ion of a replica becomes one subspecies of its
// combined ion (Sec. II D), one thread per record slot of a cell
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ungroup(const Replica* rep, int buf, const uint32_t* prefix, double fsp,
                                                 double fop, double fsm, double fom, uint32_t draw_lo,
                                                 uint32_t draw_hi, int8_t* labels, unsigned long long* counts)
{
    const Replica& R = *rep;
    const uint32_t c = blockIdx.x;
    const uint32_t nc = R.cnt[buf][c];
    __shared__ unsigned int cnt[6];
    if (threadIdx.x < 6) cnt[threadIdx.x] = 0u;
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < nc; j += blockDim.x) {
        const uint32_t meta = R.rec[buf][(size_t)c * R.cap + j].w;
        const uint32_t i = prefix[c] + j; // the particle's index in the library's order
        int8_t lab = 0;
        if (rec_is_ion(meta)) {
            uint32_t w[4];
            philox4x32_10(draw_lo, draw_hi, i, TAG_UNGROUP, R.key0, R.key1, w);
            const double u = unit53(w[0], w[1]);
            const int neg = (meta & 7u) == KIND_XNEG;
            const double fs = neg ? fsm : fsp, fo = neg ? fom : fop;
            lab = (int8_t)(u < fs ? 1 : (u < fs + fo ? 2 : 3));
            atomicAdd(&cnt[3 * neg + lab - 1], 1u);
        }
        if (labels) labels[i] = lab;
    }
    __syncthreads();
    if (threadIdx.x < 6 && cnt[threadIdx.x]) atomicAdd(&counts[threadIdx.x], (unsigned long long)cnt[threadIdx.x]);
}

hipError_t launch_ungroup(const Replica* rep_dev, const Replica& rep_host, int buf, const uint32_t* prefix,
                          const double frac[4], uint64_t draw, int8_t* labels, unsigned long long* counts,
                          hipStream_t s)
{
    hipLaunchKernelGGL(k_ungroup, dim3(rep_host.ncells), dim3(256), 0, s, rep_dev, buf, prefix, frac[0], frac[1],
                       frac[2], frac[3], (uint32_t)draw, (uint32_t)(draw >> 32), labels, counts);
    return hipGetLastError();
}

// ------------------------------------------------------------------------
// k_energy: total energy of one replica from scratch, FP64, one wave per cell
// ------------------------------------------------------------------------
__device__ double pair_energy_full(const uint4& a, const uint4& b, double scale, uint64_t R2, double lB,
                                   double kappa, double eps, int ion_coupling)
{
    const int ia = rec_is_ion(a.w), ib = rec_is_ion(b.w);
    if (!ion_coupling && (ia || ib)) return 0.0;
    const int32_t dx = (int32_t)(b.x - a.x), dy = (int32_t)(b.y - a.y), dz = (int32_t)(b.z - a.z);
    const uint32_t ax = (uint32_t)abs(dx), ay = (uint32_t)abs(dy), az = (uint32_t)abs(dz);
    const uint64_t r2i = (uint64_t)ax * ax + (uint64_t)ay * ay + (uint64_t)az * az;
    const double r2 = (double)r2i * scale * scale;
    double e = 0.0;
    if (eps > 0.0 && (ia || ib) && r2 < 1.2599210498948731647672106) {
        if (r2 < 0.25) return __longlong_as_double(0x7FF0000000000000ll);
        const double ir2 = 1.0 / r2, ir6 = ir2 * ir2 * ir2;
        e += 4.0 * eps * (ir6 * ir6 - ir6) + eps;
    }
    const int qa = rec_q(a.w), qb = rec_q(b.w);
    if (r2i < R2 && qa != 0 && qb != 0) {
        const double r = sqrt(r2);
        e += lB * (double)(qa * qb) * exp(-kappa * r) / r;
    }
    return e;
}

__global__ __launch_bounds__(64) void k_energy(const Replica* rep, int buf, double lB, double eps, int ion_coupling,
                                               double* out)
{
    const Replica& R = *rep;
    const uint32_t n = R.n, cap = R.cap;
    const uint32_t c = blockIdx.x;
    const uint32_t cx = c % n, cy = (c / n) % n, cz = c / (n * n);
    const uint4* recb = R.rec[buf];
    const uint32_t* cntb = R.cnt[buf];
    const uint32_t nc = cntb[c];
    double acc = 0.0;
    for (uint32_t i = threadIdx.x; i < nc; i += 64) {
        const uint4 a = recb[(size_t)c * cap + i];
        for (int o = 0; o < 27; ++o) {
            const uint32_t x = (cx + n + (uint32_t)(o % 3) - 1u) % n, y = (cy + n + (uint32_t)((o / 3) % 3) - 1u) % n,
                           z = (cz + n + (uint32_t)(o / 9) - 1u) % n;
            const uint32_t oc = x + n * (y + n * z);
            const uint32_t m = cntb[oc];
            for (uint32_t j = 0; j < m; ++j) {
                if (oc == c && j == i) continue;
                acc += 0.5 * pair_energy_full(a, recb[(size_t)oc * cap + j], R.scale, R.R2, lB, R.kappa, eps,
                                              ion_coupling);
            }
        }
        if (rec_is_ion(a.w) && ion_coupling && eps > 0.0) {
            for (uint32_t k = 0; k < R.ncores; ++k) {
                const uint4 cc = R.core_x[k];
                const int32_t dx = (int32_t)(cc.x - a.x), dy = (int32_t)(cc.y - a.y), dz = (int32_t)(cc.z - a.z);
                const double fx = dx * R.scale, fy = dy * R.scale, fz = dz * R.scale;
                const double rr = sqrt(fx * fx + fy * fy + fz * fz);
                const double sh = rr - R.core_delta[k];
                if (sh < 1.122462048309373) {
                    if (sh < 0.5) { acc += __longlong_as_double(0x7FF0000000000000ll); continue; }
                    const double ir2 = 1.0 / (sh * sh), ir6 = ir2 * ir2 * ir2;
                    acc += 4.0 * eps * (ir6 * ir6 - ir6) + eps;
                }
            }
        }
    }
    acc = wave_sum(acc);
    if (threadIdx.x == 0) out[c] = acc;
}

__global__ void k_philox(int64_t n, const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t w[4];
    philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3], k0, k1, w);
    for (int k = 0; k < 4; ++k) out[4 * i + k] = w[k];
}

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------
hipError_t launch_bin(const SweepArgs& a, hipStream_t s)
{
    const uint32_t per = BIN_THREADS / 64 * (uint32_t)a.bin_cpw;
    if (a.bin_dense_any)
        hipLaunchKernelGGL(k_bin, dim3((a.ncell_total + per - 1) / per), dim3(BIN_THREADS), 0, s, a);
    if (a.bin_sparse_any)
        hipLaunchKernelGGL(k_bin_sparse, dim3((a.ncell_total + BIN_THREADS - 1) / BIN_THREADS), dim3(BIN_THREADS), 0,
                           s, a);
    return hipGetLastError();
}

hipError_t launch_plan(const SweepArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_plan, dim3((a.ndom_total + 63u) / 64u, 8), dim3(64), 0, s, a);
    return hipGetLastError();
}

template <typename Real, bool LEARNED, bool RELOC>
static void launch_phase_f(const SweepArgs& a, dim3 grid, dim3 block, size_t lds, hipStream_t s)
{
    if (!LEARNED && a.bin_sparse_any) hipLaunchKernelGGL((k_phase_fast<Real, RELOC>), grid, block, lds, s, a);
    else if (LEARNED && sizeof(Real) == 4) hipLaunchKernelGGL((k_phase_learned32<RELOC>), grid, block, lds, s, a);
    else hipLaunchKernelGGL((k_phase<Real, LEARNED, RELOC>), grid, block, lds, s, a);
}

template <typename Real, bool LEARNED>
static void launch_phase_r(const SweepArgs& a, dim3 grid, dim3 block, size_t lds, hipStream_t s)
{
    if (a.ion_trials > 0) launch_phase_f<Real, LEARNED, true>(a, grid, block, lds, s);
    else launch_phase_f<Real, LEARNED, false>(a, grid, block, lds, s);
}

hipError_t launch_phase(const SweepArgs& a, size_t lds, hipStream_t s)
{
    const dim3 grid(a.ndom_total), block(PHASE_THREADS);
    if (a.precision == 64) {
        if (a.learned) launch_phase_r<double, true>(a, grid, block, lds, s);
        else launch_phase_r<double, false>(a, grid, block, lds, s);
    } else {
        if (a.learned) launch_phase_r<float, true>(a, grid, block, lds, s);
        else launch_phase_r<float, false>(a, grid, block, lds, s);
    }
    return hipGetLastError();
}

hipError_t launch_sweep_end(const SweepArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_sweep_end, dim3((a.nrep + 3u) / 4u), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_sweep_advance, dim3(1), dim3(64), 0, s, a);
    return hipGetLastError();
}

// Fixed device scratch of the energy entry point that allocates nothing: the
// replica's descriptor in its first NOALLOC_DESC_BYTES, then one FP64 sum per
// cell for at most NOALLOC_CELLS cells (8 MiB + 1 KiB per device, held until
// the process ends).  Host code never passes the symbol itself to a kernel or
// a copy: noalloc_scratch() resolves its address on the current device once
// and hands out that pointer.
static __device__ __align__(256) unsigned char scratch[NOALLOC_DESC_BYTES + NOALLOC_CELLS * sizeof(double)];

static_assert(sizeof(Replica) <= NOALLOC_DESC_BYTES, "the descriptor slot holds a replica descriptor");

hipError_t noalloc_scratch(void** out)
{
    static std::mutex mu;
    static void* ptr[NOALLOC_MAX_DEVICES] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[dev] = p;
    }
    *out = ptr[dev];
    return hipSuccess;
}

hipError_t launch_energy(const Replica* rep_dev, const Replica& rep_host, double lB, double eps, int ion_coupling,
                         int buf, double* out_per_cell, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy, dim3(rep_host.ncells), dim3(64), 0, s, rep_dev, buf, lB, eps, ion_coupling,
                       out_per_cell);
    return hipGetLastError();
}

hipError_t launch_philox(int64_t n, const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(k_philox, dim3((uint32_t)blocks), dim3(256), 0, s, n, ctr, k0, k1, out);
    return hipGetLastError();
}

hipError_t set_phase_lds_limit(size_t bytes)
{
    const void* fns[] = {(const void*)k_phase<float, false, false>, (const void*)k_phase<double, false, false>,
                         (const void*)k_phase<float, true, false>,  (const void*)k_phase<double, true, false>,
                         (const void*)k_phase<float, false, true>,  (const void*)k_phase<double, false, true>,
                         (const void*)k_phase<float, true, true>,   (const void*)k_phase<double, true, true>,
                         (const void*)k_phase_fast<float, false>,   (const void*)k_phase_fast<double, false>,
                         (const void*)k_phase_fast<float, true>,    (const void*)k_phase_fast<double, true>,
                         (const void*)k_phase_learned32<false>,     (const void*)k_phase_learned32<true>};
    for (const void* f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

} // namespace crmc

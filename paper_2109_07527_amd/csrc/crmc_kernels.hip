// CDNA4 (gfx950) kernels of the CR-MC hot path.
//
//   k_bin        per sweep: draw the grid shift, re-bin every record into the
//                shifted cells (stable: old cell order, then order in the old
//                cell), sample per-site occupancy.  One wavefront per new cell,
//                gathering from the (at most 27, usually 8) old cells that
//                overlap it, so no atomics and no scan are needed.
//   k_phase<R>   per colour: one 256-thread workgroup per domain (one cell, or
//                two reflection-paired cells of the colour).  Stages the
//                domain's cells and their 26-cell neighbourhoods in LDS, then
//                runs the domain's trials back to back: Philox words, move and
//                participants, pair sum of the energy change over the staged
//                records (R = float or double terms, FP64 accumulation,
//                wavefront + workgroup reduction), acceptance of Sec. II C,
//                commit in LDS.  Writes the cells back at the end.
//   k_sweep_end  per sweep: series row, group histograms, sweep counter.
//   k_energy     total energy of a replica from scratch (FP64), per cell.
#include "crmc_internal.h"

#include <math.h>

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
// integer helpers shared by all kernels
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

// cell boundary b_k = ceil(k 2^32 / n) (b_n = 2^32)
__device__ __forceinline__ uint64_t cell_lo(uint32_t k, uint32_t n)
{
    return (((uint64_t)k << 32) + (uint64_t)n - 1u) / (uint64_t)n;
}
__device__ __forceinline__ uint32_t cell_of(uint32_t y, uint32_t n) { return __umulhi(y, n); }

__device__ __forceinline__ void grid_shift(const Replica& R, uint64_t sweep, int fixed, uint32_t o[3])
{
    if (fixed) { o[0] = o[1] = o[2] = 0u; return; }
    uint32_t w[4];
    philox4x32_10((uint32_t)sweep, 0u, 0u, TAG_SHIFT, R.key0, R.key1, w);
    o[0] = w[0]; o[1] = w[1]; o[2] = w[2];
}

__device__ __forceinline__ int rec_kind(uint32_t meta) { return (int)(meta & 7u); }
__device__ __forceinline__ int rec_charged(uint32_t meta) { return (int)((meta >> 3) & 1u); }
__device__ __forceinline__ int rec_is_ion(uint32_t meta)
{
    const uint32_t k = meta & 7u;
    return k == KIND_XPOS || k == KIND_XNEG;
}
__device__ __forceinline__ int rec_q(uint32_t meta)
{
    const uint32_t k = meta & 7u, c = (meta >> 3) & 1u;
    if (k == KIND_ACID) return -(int)c;
    if (k == KIND_BASE) return (int)c;
    if (k == KIND_XPOS) return 1;
    if (k == KIND_XNEG) return -1;
    return 0;
}

// replica owning a flattened index, by binary search on a prefix field
template <int FIELD>
__device__ __forceinline__ uint32_t find_replica(const Replica* reps, uint32_t nrep, uint32_t x)
{
    uint32_t lo = 0, hi = nrep; // invariant: prefix(lo) <= x < prefix(hi)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        const uint32_t p = FIELD == 0 ? reps[mid].cell_begin : reps[mid].dom_begin;
        if (p <= x) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const uint32_t lane = threadIdx.x & 63u;
    return lane ? (~0ull >> (64u - lane)) : 0ull;
}

// ------------------------------------------------------------------------
// k_bin: stable re-binning into the shifted grid of this sweep
// ------------------------------------------------------------------------
__global__ __launch_bounds__(BIN_THREADS) void k_bin(SweepArgs a)
{
    const uint32_t gcell = blockIdx.x;
    const uint32_t r = find_replica<0>(a.reps, a.nrep, gcell);
    const Replica& R = a.reps[r];
    const uint32_t n = R.n, cap = R.cap;
    const uint32_t k = gcell - R.cell_begin;
    const uint64_t s = *a.sweep;
    const int cur = (int)(s & 1u), nxt = cur ^ 1;
    const uint4* __restrict__ src = R.rec[cur];
    const uint32_t* __restrict__ scnt = R.cnt[cur];
    uint4* __restrict__ dst = R.rec[nxt];

    uint32_t on[3], oo[3];
    grid_shift(R, s, a.fixed_grid, on);
    if (s == 0) { oo[0] = oo[1] = oo[2] = 0u; }
    else grid_shift(R, s - 1, a.fixed_grid, oo);

    const uint32_t kc[3] = {k % n, (k / n) % n, k / (n * n)};
    uint32_t cand[3][3];
    int ncand[3];
    for (int d = 0; d < 3; ++d) {
        const uint32_t lo_abs = on[d] + (uint32_t)cell_lo(kc[d], n);
        const uint32_t hi_abs = on[d] + (uint32_t)(cell_lo(kc[d] + 1, n) - 1u);
        const uint32_t j0 = cell_of(lo_abs - oo[d], n), j1 = cell_of(hi_abs - oo[d], n);
        const int m = (int)((j1 + n - j0) % n) + 1;
        uint32_t v[3];
        for (int i = 0; i < m; ++i) v[i] = (j0 + (uint32_t)i) % n;
        // ascending (wrap-around puts small indices last)
        for (int i = 0; i < m; ++i)
            for (int j = i + 1; j < m; ++j)
                if (v[j] < v[i]) { uint32_t t = v[i]; v[i] = v[j]; v[j] = t; }
        for (int i = 0; i < m; ++i) cand[d][i] = v[i];
        ncand[d] = m;
    }

    const uint64_t lt = lanemask_lt();
    const uint32_t lane = threadIdx.x;
    uint32_t base = 0;
    for (int iz = 0; iz < ncand[2]; ++iz)
        for (int iy = 0; iy < ncand[1]; ++iy)
            for (int ix = 0; ix < ncand[0]; ++ix) {
                const uint32_t oc = cand[0][ix] + n * (cand[1][iy] + n * cand[2][iz]);
                const uint32_t cc = scnt[oc];
                for (uint32_t b = 0; b < cc; b += 64u) {
                    const uint32_t i = b + lane;
                    bool match = false;
                    uint4 rec = make_uint4(0, 0, 0, 0);
                    if (i < cc) {
                        rec = src[(size_t)oc * cap + i];
                        match = cell_of(rec.x - on[0], n) == kc[0] && cell_of(rec.y - on[1], n) == kc[1] &&
                                cell_of(rec.z - on[2], n) == kc[2];
                    }
                    const uint64_t mask = __ballot(match);
                    if (match) {
                        const uint32_t pos = base + (uint32_t)__popcll(mask & lt);
                        if (pos < cap) dst[(size_t)k * cap + pos] = rec;
                        const uint32_t sid = rec.w >> 8;
                        if (sid != NO_SITE && rec_charged(rec.w)) R.occupancy[sid] += 1u;
                    }
                    base += (uint32_t)__popcll(mask);
                }
            }
    if (lane == 0) {
        R.cnt[nxt][k] = base < cap ? base : cap;
        if (base > cap) atomicOr(a.err, ERR_BIN_CAPACITY);
    }
}

// ------------------------------------------------------------------------
// precision policy of the pair terms
// ------------------------------------------------------------------------
template <typename Real> struct Math;
template <> struct Math<float> {
    __device__ static __forceinline__ float rsqrt(float x) { return rsqrtf(x); }
    __device__ static __forceinline__ float ex(float x) { return __expf(x); }
    __device__ static __forceinline__ float rcp(float x) { return __frcp_rn(x); }
    __device__ static __forceinline__ float sqrt_(float x) { return sqrtf(x); }
};
template <> struct Math<double> {
    __device__ static __forceinline__ double rsqrt(double x) { return 1.0 / sqrt(x); }
    __device__ static __forceinline__ double ex(double x) { return exp(x); }
    __device__ static __forceinline__ double rcp(double x) { return 1.0 / x; }
    __device__ static __forceinline__ double sqrt_(double x) { return sqrt(x); }
};

// a particle whose state the trial changes
struct Chg {
    uint32_t x, y, z;
    int dq;     // charge change seen by every other particle
    int dw;     // +1 inserted free ion, -1 deleted free ion, 0 otherwise
    int member; // domain cell it lives in
    int own;    // index in that cell's list, -1 if inserted
    int q_old, q_new, ion, pres_old, pres_new;
};

struct PairParams {
    float scale_f;
    double scale_d;
    uint64_t R2;
    double lB, kappa, eps;
    int ion_coupling;
};

template <typename Real>
__device__ __forceinline__ double pair_term(const uint4& rec, const Chg& c, const PairParams& P, int& ov)
{
    const int ionj = rec_is_ion(rec.w);
    if (!P.ion_coupling && ionj) return 0.0;
    const int qj = rec_q(rec.w);
    const bool coul = c.dq != 0 && qj != 0;
    const bool ev = c.dw != 0;
    if (!coul && !ev) return 0.0;
    const int32_t dx = (int32_t)(rec.x - c.x), dy = (int32_t)(rec.y - c.y), dz = (int32_t)(rec.z - c.z);
    const Real sc = sizeof(Real) == 4 ? (Real)P.scale_f : (Real)P.scale_d;
    const Real fx = (Real)dx * sc, fy = (Real)dy * sc, fz = (Real)dz * sc;
    const Real r2 = fx * fx + fy * fy + fz * fz;
    double e = 0.0;
    if (coul) {
        const uint32_t ax = (uint32_t)abs(dx), ay = (uint32_t)abs(dy), az = (uint32_t)abs(dz);
        const uint64_t r2i = (uint64_t)ax * ax + (uint64_t)ay * ay + (uint64_t)az * az;
        if (r2i < P.R2) {
            const Real rinv = Math<Real>::rsqrt(r2);
            const Real r = r2 * rinv;
            const Real phi = Math<Real>::ex(-(Real)P.kappa * r) * rinv;
            e += P.lB * (double)(c.dq * qj) * (double)phi;
        }
    }
    if (ev && r2 < (Real)1.2599210498948731647672106) {
        if (r2 < (Real)0.25) {
            if (c.dw > 0) ov = 1;
        } else {
            const Real ir2 = Math<Real>::rcp(r2);
            const Real ir6 = ir2 * ir2 * ir2;
            const Real w = (Real)4.0 * (Real)P.eps * (ir6 * ir6 - ir6) + (Real)P.eps;
            e += (double)c.dw * (double)w;
        }
    }
    return e;
}

template <typename Real>
__device__ __forceinline__ double wca_core(const Chg& c, const uint4& cx, double delta, const PairParams& P, int& ov)
{
    const int32_t dx = (int32_t)(cx.x - c.x), dy = (int32_t)(cx.y - c.y), dz = (int32_t)(cx.z - c.z);
    const Real sc = sizeof(Real) == 4 ? (Real)P.scale_f : (Real)P.scale_d;
    const Real fx = (Real)dx * sc, fy = (Real)dy * sc, fz = (Real)dz * sc;
    const Real r = Math<Real>::sqrt_(fx * fx + fy * fy + fz * fz);
    const Real sh = r - (Real)delta;
    if (!(sh < (Real)1.122462048309373)) return 0.0;
    if (sh < (Real)0.5) {
        if (c.dw > 0) ov = 1;
        return 0.0;
    }
    const Real ir2 = Math<Real>::rcp(sh * sh);
    const Real ir6 = ir2 * ir2 * ir2;
    return (double)c.dw * (double)((Real)4.0 * (Real)P.eps * (ir6 * ir6 - ir6) + (Real)P.eps);
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ------------------------------------------------------------------------
// k_phase: one colour of one sweep
// ------------------------------------------------------------------------
struct PhaseShared {
    int32_t pre[53];       // prefix of the 52 neighbour segments (member 0, then 1)
    uint32_t seg_cell[52]; // neighbour cell of each segment
    double red[2][4];
    int32_t ovf[2][4];
    uint32_t att[6], acc[6];
    int32_t dtot[4];
};

// record g of the neighbour list of the domain (concatenated over both members)
__device__ __forceinline__ uint4 neighbour_global(const PhaseShared& S, const uint4* recb, uint32_t cap, int g)
{
    int q = 0;
    while (S.pre[q + 1] <= g) ++q;
    return recb[(size_t)S.seg_cell[q] * cap + (uint32_t)(g - S.pre[q])];
}

// k-th record of the domain (member 0's list, then member 1's) matching the
// predicate; every wavefront computes the same answer independently
template <typename Pred>
__device__ __forceinline__ int domain_kth(const uint4* own0, int n0, const uint4* own1, int n1, Pred pred, int k)
{
    const int lane = threadIdx.x & 63;
    const uint64_t lt = lanemask_lt();
    const int total = n0 + n1;
    for (int b = 0; b < total; b += 64) {
        const int g = b + lane;
        bool p = false;
        if (g < total) p = pred(g < n0 ? own0[g].w : own1[g - n0].w);
        const uint64_t mask = __ballot(p);
        const int cnt = __popcll(mask);
        if (k < cnt) {
            const bool mine = p && __popcll(mask & lt) == k;
            const uint64_t hit = __ballot(mine);
            return b + (__ffsll((long long)hit) - 1);
        }
        k -= cnt;
    }
    return -1;
}

__device__ __forceinline__ int domain_count(const uint4* own0, int n0, const uint4* own1, int n1, int kind, int charged)
{
    const int lane = threadIdx.x & 63;
    const int total = n0 + n1;
    int c = 0;
    for (int b = 0; b < total; b += 64) {
        const int g = b + lane;
        bool p = false;
        if (g < total) {
            const uint32_t m = g < n0 ? own0[g].w : own1[g - n0].w;
            p = rec_kind(m) == kind && (kind == (int)KIND_XPOS || kind == (int)KIND_XNEG || rec_charged(m) == charged);
        }
        c += __popcll(__ballot(p));
    }
    return c;
}

template <typename Real>
__global__ __launch_bounds__(PHASE_THREADS) void k_phase(SweepArgs a)
{
    extern __shared__ uint4 smem[];
    __shared__ PhaseShared S;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t gd = blockIdx.x;
    const uint32_t r = find_replica<1>(a.reps, a.nrep, gd);
    const Replica& R = a.reps[r];
    const uint32_t n = R.n, h = R.h, cap = R.cap;
    const uint64_t s = *a.sweep;
    const int buf = (int)((s + 1u) & 1u);
    uint4* __restrict__ recb = R.rec[buf];
    uint32_t* __restrict__ cntb = R.cnt[buf];
    const int colour = a.colour;
    const uint32_t px = colour & 1, py = (colour >> 1) & 1, pz = (colour >> 2) & 1;

    // ---- the domain of this workgroup -------------------------------------
    const uint32_t M = h * h * h;
    const uint32_t d = gd - R.dom_begin;
    uint32_t ma, mb;
    if (a.pairing) {
        uint32_t w[4];
        philox4x32_10((uint32_t)s, (uint32_t)colour, 0u, TAG_PAIR, R.key0, R.key1, w);
        const uint32_t rr = pick32(w[0], M);
        const uint32_t c = (uint32_t)(((uint64_t)M - 1u + 2ull * M - 2ull * rr) % M);
        const uint32_t half = c >> 1;
        if (d <= half) { ma = d; mb = c - d; }
        else { ma = c + 1u + (d - half - 1u); mb = M + c - ma; }
    } else {
        ma = mb = d;
    }
    const int ncell = (ma == mb) ? 1 : 2;
    uint32_t cellv[2], cc[2][3];
    {
        const uint32_t mm[2] = {ma, mb};
        for (int j = 0; j < 2; ++j) {
            const uint32_t m = mm[j];
            cc[j][0] = 2u * (m % h) + px;
            cc[j][1] = 2u * ((m / h) % h) + py;
            cc[j][2] = 2u * (m / (h * h)) + pz;
            cellv[j] = cc[j][0] + n * (cc[j][1] + n * cc[j][2]);
        }
    }

    // LDS pool of a.budget records: each member's list, with room for the
    // growth its trials can cause (two ions per trial), then the neighbours
    const int ntr = a.trials * ncell;
    int n_own[2];
    n_own[0] = (int)cntb[cellv[0]];
    n_own[1] = ncell == 2 ? (int)cntb[cellv[1]] : 0;
    const int room0 = min((int)cap, n_own[0] + 2 * ntr);
    const int room1 = ncell == 2 ? min((int)cap, n_own[1] + 2 * ntr) : 0;
    uint4* own0 = smem;
    uint4* own1 = smem + room0;
    uint4* nb = smem + room0 + room1;

    // ---- neighbour segments and staging ------------------------------------
    if (tid < 52) {
        const int j = tid / 26, q = tid % 26;
        const int o = q < 13 ? q : q + 1;
        const int dxo = o % 3 - 1, dyo = (o / 3) % 3 - 1, dzo = o / 9 - 1;
        uint32_t nc = 0, cnt = 0;
        if (j < ncell) {
            const uint32_t x = (cc[j][0] + n + (uint32_t)dxo) % n, y = (cc[j][1] + n + (uint32_t)dyo) % n,
                           z = (cc[j][2] + n + (uint32_t)dzo) % n;
            nc = x + n * (y + n * z);
            cnt = cntb[nc];
        }
        S.seg_cell[tid] = nc;
        S.pre[tid + 1] = (int32_t)cnt;
    }
    if (tid < 6) { S.att[tid] = 0; S.acc[tid] = 0; }
    if (tid < 4) S.dtot[tid] = 0;
    __syncthreads();
    if (tid == 0) {
        S.pre[0] = 0;
        for (int q = 0; q < 52; ++q) S.pre[q + 1] += S.pre[q];
    }
    for (int i = tid; i < n_own[0]; i += PHASE_THREADS) own0[i] = recb[(size_t)cellv[0] * cap + i];
    for (int i = tid; i < n_own[1]; i += PHASE_THREADS) own1[i] = recb[(size_t)cellv[1] * cap + i];
    __syncthreads();
    const int nb_total = S.pre[52];
    const bool staged = room0 + room1 + nb_total <= a.budget;
    if (staged) {
        for (int g = tid; g < nb_total; g += PHASE_THREADS) {
            int lo = 0, hi = 52; // pre[lo] <= g < pre[hi]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (S.pre[mid] <= g) lo = mid; else hi = mid;
            }
            nb[g] = recb[(size_t)S.seg_cell[lo] * cap + (uint32_t)(g - S.pre[lo])];
        }
    } else if (tid == 0) {
        atomicOr(a.err, INFO_UNSTAGED);
    }
    __syncthreads();
    const int nb_begin[2] = {S.pre[0], S.pre[26]};
    const int nb_count[2] = {S.pre[26] - S.pre[0], S.pre[52] - S.pre[26]};

    // ---- static move set and counts of the domain ---------------------------
    int m0a = domain_count(own0, n_own[0], own1, n_own[1], KIND_ACID, 0);
    int mca = domain_count(own0, n_own[0], own1, n_own[1], KIND_ACID, 1);
    int m0b = domain_count(own0, n_own[0], own1, n_own[1], KIND_BASE, 0);
    int mcb = domain_count(own0, n_own[0], own1, n_own[1], KIND_BASE, 1);
    int npos = domain_count(own0, n_own[0], own1, n_own[1], KIND_XPOS, 1);
    int nneg = domain_count(own0, n_own[0], own1, n_own[1], KIND_XNEG, 1);
    int react[3], nreact = 0;
    if (m0a + mca > 0) react[nreact++] = 0;
    if (m0b + mcb > 0) react[nreact++] = 1;
    react[nreact++] = 2;

    // insertion regions and volume terms of the members
    uint32_t on[3];
    grid_shift(R, s, a.fixed_grid, on);
    uint32_t ins_base[2][3], ins_w[2][3];
    double lnZ[2];
    for (int j = 0; j < ncell; ++j) {
        double lnV = 0.0;
        for (int dd = 0; dd < 3; ++dd) {
            const uint64_t lo = cell_lo(cc[j][dd], n), hi = cell_lo(cc[j][dd] + 1u, n);
            ins_base[j][dd] = on[dd] + (uint32_t)lo;
            ins_w[j][dd] = (uint32_t)(hi - lo);
            lnV += log((double)(hi - lo));
        }
        lnZ[j] = (R.lnZ0 + log((double)ncell)) + lnV;
    }

    PairParams P;
    P.scale_f = (float)R.scale;
    P.scale_d = R.scale;
    P.R2 = R.R2;
    P.lB = a.lB;
    P.kappa = R.kappa;
    P.eps = a.eps;
    P.ion_coupling = a.ion_coupling;
    const bool ev_on = a.eps > 0.0 && a.ion_coupling;

    double dE = 0.0;
    for (int t = 0; t < ntr; ++t) {
        // 20 Philox words: lane b of every wavefront computes block b
        uint32_t wl[4];
        philox4x32_10((uint32_t)s, cellv[0], (uint32_t)t * 8u + (uint32_t)(lane < 5 ? lane : 0), TAG_TRIAL,
                      R.key0, R.key1, wl);
        uint32_t W[20];
#pragma unroll
        for (int i = 0; i < 20; ++i) W[i] = (uint32_t)__builtin_amdgcn_readlane((int)wl[i & 3], i >> 2);

        const uint32_t kk = pick32(W[0], (uint32_t)(2 * nreact));
        const int move = 2 * react[kk >> 1] + (int)(kk & 1u);
        int auto_reject = 0, site = -1, del_pos = -1, del_neg = -1, ins_pos = 0, ins_neg = 0;
        double lnp_counts = 0.0;
        const uint4* o0 = own0;
        const uint4* o1 = own1;
        const int n0 = n_own[0], n1 = n_own[1];
        switch (move) {
        case 0:
            if (m0a == 0) { auto_reject = 1; break; }
            site = domain_kth(o0, n0, o1, n1, [](uint32_t m) { return rec_kind(m) == (int)KIND_ACID && !rec_charged(m); },
                              (int)pick32(W[1], (uint32_t)m0a));
            ins_pos = 1;
            lnp_counts = log((double)m0a) - log((double)(mca + 1)) - log((double)(npos + 1)) + R.lnKA;
            break;
        case 1:
            if (mca == 0 || npos == 0) { auto_reject = 1; break; }
            site = domain_kth(o0, n0, o1, n1, [](uint32_t m) { return rec_kind(m) == (int)KIND_ACID && rec_charged(m); },
                              (int)pick32(W[1], (uint32_t)mca));
            del_pos = domain_kth(o0, n0, o1, n1, [](uint32_t m) { return rec_kind(m) == (int)KIND_XPOS; },
                                 (int)pick32(W[2], (uint32_t)npos));
            lnp_counts = log((double)mca) + log((double)npos) - log((double)(m0a + 1)) - R.lnKA;
            break;
        case 2:
            if (m0b == 0) { auto_reject = 1; break; }
            site = domain_kth(o0, n0, o1, n1, [](uint32_t m) { return rec_kind(m) == (int)KIND_BASE && !rec_charged(m); },
                              (int)pick32(W[1], (uint32_t)m0b));
            ins_neg = 1;
            lnp_counts = log((double)m0b) - log((double)(mcb + 1)) - log((double)(nneg + 1)) + R.lnKB;
            break;
        case 3:
            if (mcb == 0 || nneg == 0) { auto_reject = 1; break; }
            site = domain_kth(o0, n0, o1, n1, [](uint32_t m) { return rec_kind(m) == (int)KIND_BASE && rec_charged(m); },
                              (int)pick32(W[1], (uint32_t)mcb));
            del_neg = domain_kth(o0, n0, o1, n1, [](uint32_t m) { return rec_kind(m) == (int)KIND_XNEG; },
                                 (int)pick32(W[3], (uint32_t)nneg));
            lnp_counts = log((double)mcb) + log((double)nneg) - log((double)(m0b + 1)) - R.lnKB;
            break;
        case 4:
            ins_pos = ins_neg = 1;
            lnp_counts = -log((double)(npos + 1)) - log((double)(nneg + 1)) + R.lnKion;
            break;
        default:
            if (npos == 0 || nneg == 0) { auto_reject = 1; break; }
            del_pos = domain_kth(o0, n0, o1, n1, [](uint32_t m) { return rec_kind(m) == (int)KIND_XPOS; },
                                 (int)pick32(W[2], (uint32_t)npos));
            del_neg = domain_kth(o0, n0, o1, n1, [](uint32_t m) { return rec_kind(m) == (int)KIND_XNEG; },
                                 (int)pick32(W[3], (uint32_t)nneg));
            lnp_counts = log((double)npos) + log((double)nneg) - R.lnKion;
            break;
        }
        const double u = unit53(W[16], W[17]);
        if (tid == 0) S.att[move] += 1u;
        if (auto_reject) {
            if (tid == 0 && a.log) {
                const unsigned long long li = atomicAdd(a.log_n, 1ull);
                if (li < a.log_cap) {
                    TrialRec& L = a.log[li];
                    L.sweep = (int64_t)s; L.cell = cellv[0]; L.trial = t; L.replica = (int32_t)r;
                    L.move = move; L.status = 2;
                    L.dU = __longlong_as_double(0x7FF8000000000000ll); L.lnp = L.dU; L.u = u;
                }
            }
            continue;
        }

        // ---- changed particles --------------------------------------------
        Chg ch[2];
        int nch = 0;
        double lnvol = 0.0;
        int ins_into[2] = {0, 0}, del_from[2] = {0, 0};
        if (site >= 0) {
            Chg& c = ch[nch++];
            c.member = site < n0 ? 0 : 1;
            c.own = site < n0 ? site : site - n0;
            const uint4 rc = (c.member ? o1 : o0)[c.own];
            c.x = rc.x; c.y = rc.y; c.z = rc.z;
            const int kind = rec_kind(rc.w), chg = rec_charged(rc.w);
            c.q_old = kind == (int)KIND_ACID ? -chg : chg;
            c.q_new = kind == (int)KIND_ACID ? -(1 - chg) : (1 - chg);
            c.dq = c.q_new - c.q_old;
            c.dw = 0; c.ion = 0; c.pres_old = 1; c.pres_new = 1;
        }
        if (del_pos >= 0 || del_neg >= 0) {
            const int dels[2] = {del_pos, del_neg};
            for (int i = 0; i < 2; ++i) {
                if (dels[i] < 0) continue;
                Chg& c = ch[nch++];
                c.member = dels[i] < n0 ? 0 : 1;
                c.own = dels[i] < n0 ? dels[i] : dels[i] - n0;
                const uint4 rc = (c.member ? o1 : o0)[c.own];
                c.x = rc.x; c.y = rc.y; c.z = rc.z;
                c.q_old = i == 0 ? 1 : -1; c.q_new = 0;
                c.ion = 1; c.pres_old = 1; c.pres_new = 0;
                c.dq = a.ion_coupling ? -c.q_old : 0;
                c.dw = ev_on ? -1 : 0;
                lnvol -= lnZ[c.member];
                del_from[c.member]++;
            }
        }
        if (ins_pos || ins_neg) {
            const int ins[2] = {ins_pos, ins_neg};
            for (int i = 0; i < 2; ++i) {
                if (!ins[i]) continue;
                Chg& c = ch[nch++];
                const uint32_t wc = i == 0 ? W[18] : W[19];
                const uint32_t* ws = i == 0 ? &W[4] : &W[10];
                const int j = ncell == 1 ? 0 : (int)pick32(wc, (uint32_t)ncell);
                c.member = j;
                c.own = -1;
                c.x = ins_base[j][0] + pick64(ws[0], ws[1], ins_w[j][0]);
                c.y = ins_base[j][1] + pick64(ws[2], ws[3], ins_w[j][1]);
                c.z = ins_base[j][2] + pick64(ws[4], ws[5], ins_w[j][2]);
                c.q_old = 0; c.q_new = i == 0 ? 1 : -1;
                c.ion = 1; c.pres_old = 0; c.pres_new = 1;
                c.dq = a.ion_coupling ? c.q_new : 0;
                c.dw = ev_on ? 1 : 0;
                lnvol += lnZ[j];
                ins_into[j]++;
            }
        }
        bool cap_fail = false;
        for (int j = 0; j < ncell; ++j)
            if (n_own[j] - del_from[j] + ins_into[j] > (int)cap) cap_fail = true;

        // ---- energy change: every wavefront sums a share of the records ------
        double acc = 0.0;
        int ov = 0;
        for (int j = 0; j < ncell; ++j) {
            int idx[2], m = 0;
            for (int i = 0; i < nch; ++i)
                if (ch[i].member == j) idx[m++] = i;
            if (m == 0) continue;
            const uint4* own = j ? o1 : o0;
            const int no = n_own[j];
            const int skip0 = ch[idx[0]].own, skip1 = m > 1 ? ch[idx[1]].own : -1;
            const int total = no + nb_count[j];
            for (int g = tid; g < total; g += PHASE_THREADS) {
                uint4 rc;
                if (g < no) {
                    if (g == skip0 || g == skip1) continue;
                    rc = own[g];
                } else {
                    const int q = nb_begin[j] + (g - no);
                    rc = staged ? nb[q] : neighbour_global(S, recb, cap, q);
                }
                acc += pair_term<Real>(rc, ch[idx[0]], P, ov);
                if (m > 1) acc += pair_term<Real>(rc, ch[idx[1]], P, ov);
            }
        }
        if (ev_on && R.ncores) {
            for (int k = tid; k < (int)R.ncores; k += PHASE_THREADS) {
                const uint4 cx = R.core_x[k];
                const double dl = R.core_delta[k];
                for (int i = 0; i < nch; ++i)
                    if (ch[i].dw != 0) acc += wca_core<Real>(ch[i], cx, dl, P, ov);
            }
        }
        if (tid == 0 && nch == 2 && (a.ion_coupling || (!ch[0].ion && !ch[1].ion))) {
            // the pair formed or broken between the two changed particles
            const int32_t dx = (int32_t)(ch[1].x - ch[0].x), dy = (int32_t)(ch[1].y - ch[0].y),
                          dz = (int32_t)(ch[1].z - ch[0].z);
            const uint32_t ax = (uint32_t)abs(dx), ay = (uint32_t)abs(dy), az = (uint32_t)abs(dz);
            const uint64_t r2i = (uint64_t)ax * ax + (uint64_t)ay * ay + (uint64_t)az * az;
            const Real sc = sizeof(Real) == 4 ? (Real)P.scale_f : (Real)P.scale_d;
            const Real fx = (Real)dx * sc, fy = (Real)dy * sc, fz = (Real)dz * sc;
            const Real r2 = fx * fx + fy * fy + fz * fz;
            const int dqq = ch[0].q_new * ch[1].q_new - ch[0].q_old * ch[1].q_old;
            if (dqq != 0 && r2i < P.R2) {
                const Real rinv = Math<Real>::rsqrt(r2);
                acc += P.lB * (double)dqq * (double)(Math<Real>::ex(-(Real)P.kappa * r2 * rinv) * rinv);
            }
            const int any_ion = ch[0].ion || ch[1].ion;
            const int pn = ev_on && any_ion && ch[0].pres_new && ch[1].pres_new;
            const int po = ev_on && any_ion && ch[0].pres_old && ch[1].pres_old;
            if ((pn || po) && r2 < (Real)1.2599210498948731647672106) {
                if (r2 < (Real)0.25) {
                    if (pn) ov = 1;
                } else {
                    const Real ir2 = Math<Real>::rcp(r2);
                    const Real ir6 = ir2 * ir2 * ir2;
                    acc += (double)(pn - po) * (double)((Real)4.0 * (Real)P.eps * (ir6 * ir6 - ir6) + (Real)P.eps);
                }
            }
        }
        const double wsum = wave_sum(acc);
        const int wov = __ballot(ov) != 0ull;
        const int par = t & 1;
        if (lane == 0) { S.red[par][wave] = wsum; S.ovf[par][wave] = wov; }
        __syncthreads();
        double dU = ((S.red[par][0] + S.red[par][1]) + S.red[par][2]) + S.red[par][3];
        if (S.ovf[par][0] | S.ovf[par][1] | S.ovf[par][2] | S.ovf[par][3]) dU = __longlong_as_double(0x7FF0000000000000ll);
        const double lnp = lnp_counts + lnvol - dU;
        const bool accept = !cap_fail && u < exp(lnp < 0.0 ? lnp : 0.0);
        if (cap_fail && tid == 0) atomicOr(a.err, ERR_INSERT_CAPACITY);
        if (tid == 0 && a.log) {
            const unsigned long long li = atomicAdd(a.log_n, 1ull);
            if (li < a.log_cap) {
                TrialRec& L = a.log[li];
                L.sweep = (int64_t)s; L.cell = cellv[0]; L.trial = t; L.replica = (int32_t)r;
                L.move = move; L.status = accept ? 1 : 0;
                L.dU = dU; L.lnp = lnp; L.u = u;
            }
        }
        if (!accept) continue;

        // ---- commit --------------------------------------------------------
        if (tid == 0) {
            S.acc[move] += 1u;
            dE += dU;
            uint4* ownv[2] = {own0, own1};
            if (site >= 0) {
                uint4& rc = ownv[ch[0].member][ch[0].own];
                rc.w ^= 8u;
                const uint32_t sid = rc.w >> 8;
                const int now = rec_charged(rc.w);
                const int g = R.site_group[sid];
                atomicAdd(&R.group_ionized[g], now ? 1 : -1);
                if (rec_kind(rc.w) == (int)KIND_ACID) S.dtot[0] += now ? 1 : -1;
                else S.dtot[1] += now ? 1 : -1;
            }
            // deletions: in one cell, the higher index first
            int dm[2], di[2], nd = 0;
            for (int i = 0; i < nch; ++i)
                if (ch[i].pres_old && !ch[i].pres_new) { dm[nd] = ch[i].member; di[nd] = ch[i].own; ++nd; }
            if (nd == 2 && dm[0] == dm[1] && di[1] > di[0]) {
                int t0 = di[0]; di[0] = di[1]; di[1] = t0;
            }
            for (int i = 0; i < nd; ++i) {
                uint4* L = ownv[dm[i]];
                int& cnt = n_own[dm[i]];
                L[di[i]] = L[cnt - 1];
                --cnt;
            }
            for (int i = 0; i < nch; ++i)
                if (!ch[i].pres_old && ch[i].pres_new) {
                    uint4* L = ownv[ch[i].member];
                    L[n_own[ch[i].member]++] = make_uint4(ch[i].x, ch[i].y, ch[i].z,
                                                          make_meta(ch[i].q_new > 0 ? KIND_XPOS : KIND_XNEG, 1u, NO_SITE));
                }
            if (ins_pos) S.dtot[2] += 1;
            if (ins_neg) S.dtot[3] += 1;
            if (del_pos >= 0) S.dtot[2] -= 1;
            if (del_neg >= 0) S.dtot[3] -= 1;
        } else {
            // the same count bookkeeping in every thread (registers stay uniform)
            for (int i = 0; i < nch; ++i) {
                if (ch[i].pres_old && !ch[i].pres_new) n_own[ch[i].member]--;
                if (!ch[i].pres_old && ch[i].pres_new) n_own[ch[i].member]++;
            }
        }
        switch (move) {
        case 0: m0a--; mca++; npos++; break;
        case 1: m0a++; mca--; npos--; break;
        case 2: m0b--; mcb++; nneg++; break;
        case 3: m0b++; mcb--; nneg--; break;
        case 4: npos++; nneg++; break;
        default: npos--; nneg--; break;
        }
        __syncthreads();
    }

    // ---- write the domain's cells back --------------------------------------
    __syncthreads();
    for (int i = tid; i < n_own[0]; i += PHASE_THREADS) recb[(size_t)cellv[0] * cap + i] = own0[i];
    for (int i = tid; i < n_own[1]; i += PHASE_THREADS) recb[(size_t)cellv[1] * cap + i] = own1[i];
    if (tid == 0) {
        cntb[cellv[0]] = (uint32_t)n_own[0];
        if (ncell == 2) cntb[cellv[1]] = (uint32_t)n_own[1];
        if (dE != 0.0) R.e_acc[cellv[0]] += dE;
        for (int i = 0; i < 6; ++i) {
            if (S.att[i]) atomicAdd((unsigned long long*)&R.moves[i], (unsigned long long)S.att[i]);
            if (S.acc[i]) atomicAdd((unsigned long long*)&R.moves[6 + i], (unsigned long long)S.acc[i]);
        }
        for (int i = 0; i < 4; ++i)
            if (S.dtot[i]) atomicAdd((unsigned long long*)&R.totals[i], (unsigned long long)(long long)S.dtot[i]);
    }
}

// ------------------------------------------------------------------------
// k_sweep_end: series row, group histograms, advance the sweep counter
// ------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sweep_end(SweepArgs a, int64_t series_first)
{
    const uint64_t s = *a.sweep;
    for (uint32_t r = 0; r < a.nrep; ++r) {
        const Replica& R = a.reps[r];
        if (threadIdx.x < 4 && R.series_cap > 0) {
            const int64_t row = (int64_t)(s % (uint64_t)R.series_cap);
            R.series[row * 4 + threadIdx.x] = (int32_t)R.totals[threadIdx.x];
        }
        for (uint32_t g = threadIdx.x; g < R.ngroups; g += blockDim.x)
            R.group_hist[R.group_hist_off[g] + R.group_ionized[g]] += 1;
    }
    (void)series_first;
    __syncthreads();
    if (threadIdx.x == 0) *a.sweep = s + 1u;
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
size_t phase_lds_bytes(uint32_t max_cap, int budget)
{
    (void)max_cap; // the pool holds the domain's cells and, when they fit, its neighbours
    return (size_t)budget * sizeof(uint4);
}

hipError_t launch_bin(const SweepArgs& a, hipStream_t s)
{
    hipLaunchKernelGGL(k_bin, dim3(a.ncell_total), dim3(BIN_THREADS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_phase(const SweepArgs& a, size_t lds, hipStream_t s)
{
    if (a.precision == 64)
        hipLaunchKernelGGL(k_phase<double>, dim3(a.ndom_total), dim3(PHASE_THREADS), lds, s, a);
    else
        hipLaunchKernelGGL(k_phase<float>, dim3(a.ndom_total), dim3(PHASE_THREADS), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_sweep_end(const SweepArgs& a, int64_t series_first, hipStream_t s)
{
    hipLaunchKernelGGL(k_sweep_end, dim3(1), dim3(256), 0, s, a, series_first);
    return hipGetLastError();
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

} // namespace crmc

namespace crmc {
hipError_t set_phase_lds_limit(size_t bytes)
{
    hipError_t e = hipFuncSetAttribute((const void*)k_phase<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)bytes);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_phase<double>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
} // namespace crmc

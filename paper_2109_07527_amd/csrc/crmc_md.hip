// CDNA4 (gfx950) kernels of the hybrid MD / CR-MC protocol: blocks of
// Langevin molecular dynamics of the free ions between sweeps (Sec. III:
// velocity Verlet with a Langevin thermostat, n_MD steps between blocks of MC
// steps; units sigma, kT and the ion mass, so tau = 1).  Sites and
// nanoparticle cores stay where they are.
//
//   k_md_vinit    Maxwell-Boltzmann velocities of the free ions at the start
//                 of a block (Box-Muller on Philox counter (step, cell, slot, 6)).
//   k_md_force    FP64 force on every free ion from the 27 cells around its
//                 cell (cells are at least rc wide): screened Coulomb inside
//                 the exact integer cutoff, excluded volume with every other
//                 particle, expanded excluded volume of the cores; with the
//                 Langevin drag and noise (counter (step, cell, slot, 7)) and
//                 the second half kick when asked.  The cell's neighbourhood
//                 is staged in LDS and eight lanes share each ion.  Pair
//                 terms in FP64, or in FP32 (summed in FP64) for FP32 handles.
//   k_md_drift    first half kick and drift, rounded to the position lattice.
//   k_md_rebin    the moved ions back into cells of the same grid (the grid of
//                 the last sweep), stably: a new cell gathers its records from
//                 the 27 cells around it in ascending cell index, each in slot
//                 order, with their velocities.  One wavefront per cell.
#include "crmc_internal.h"

#include <math.h>

namespace crmc {

constexpr uint32_t TAG_MDVEL = 6, TAG_MDNOISE = 7;

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the two
// multiply-xor bijections with the Weyl key schedule
__device__ __forceinline__ void md_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                          uint32_t k1, uint32_t out[4])
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

// three standard normal deviates from one Philox block (Box-Muller on the
// uniforms (w0 + 1) / 2^32, w1 / 2^32 and (w2 + 1) / 2^32, w3 / 2^32)
__device__ __forceinline__ void md_normals3(const Replica& R, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag,
                                            double z[3])
{
    uint32_t w[4];
    md_philox(c0, c1, c2, tag, R.key0, R.key1, w);
    const double TWO32 = 4294967296.0, TWO_PI = 6.283185307179586476925286766559;
    const double u1 = ((double)w[0] + 1.0) / TWO32, u2 = (double)w[1] / TWO32;
    const double u3 = ((double)w[2] + 1.0) / TWO32, u4 = (double)w[3] / TWO32;
    const double r1 = sqrt(-2.0 * log(u1)), r2 = sqrt(-2.0 * log(u3));
    z[0] = r1 * cos(TWO_PI * u2);
    z[1] = r1 * sin(TWO_PI * u2);
    z[2] = r2 * cos(TWO_PI * u4);
}

__device__ __forceinline__ int md_is_ion(uint32_t meta)
{
    const uint32_t k = meta & 7u;
    return k == KIND_XPOS || k == KIND_XNEG;
}

// charge of a record, looked up branch-free from meta & 15 (kind + 8 charged):
// two bits per value hold q + 1 (an acid -1 when charged, a base +1, a cation
// +1 and an anion -1 whatever the flag, everything else 0)
__device__ __forceinline__ int md_q(uint32_t meta)
{
    return (int)((0x54a15495u >> (2u * (meta & 15u))) & 3u) - 1;
}

// Force on ion a (charge qa) from record rb, added to f: screened Coulomb
// inside the exact integer cutoff, excluded volume below 2^(1/6), both as
// minus the gradient of the truncated pair energy, in FP64.
struct MdPair {
    double s, lB, kappa, eps; // lattice unit, Bjerrum length, screening, WCA depth
    uint64_t R2;              // Coulomb cutoff on the integer squared distance
    float sf, lBf, kappaf, klf, epsf; // FP32 copies; klf = -kappa log2(e)
};

__device__ __forceinline__ void md_pair(const uint4& ra, int qa, const uint4& rb, const MdPair& P, double f[3])
{
    const double s = P.s;
    const int32_t dx = (int32_t)(ra.x - rb.x), dy = (int32_t)(ra.y - rb.y), dz = (int32_t)(ra.z - rb.z);
    const uint32_t ax = (uint32_t)abs(dx), ay = (uint32_t)abs(dy), az = (uint32_t)abs(dz);
    const uint64_t r2i = (uint64_t)ax * ax + (uint64_t)ay * ay + (uint64_t)az * az;
    const double fx = dx * s, fy = dy * s, fz = dz * s;
    const double r2 = fx * fx + fy * fy + fz * fz;
    double g = 0.0;
    const int qb = md_q(rb.w);
    if (r2i < P.R2 && qa != 0 && qb != 0) {
        const double r = sqrt(r2);
        g += P.lB * (double)(qa * qb) * exp(-P.kappa * r) * (1.0 + P.kappa * r) / (r2 * r);
    }
    if (P.eps > 0.0 && r2 < 1.2599210498948731647672106) {
        const double ir2 = 1.0 / r2, ir6 = ir2 * ir2 * ir2;
        g += 4.0 * P.eps * (12.0 * ir6 * ir6 - 6.0 * ir6) * ir2;
    }
    f[0] += g * fx; f[1] += g * fy; f[2] += g * fz;
}

// The same force with FP32 pair arithmetic (hardware reciprocal square root,
// base-2 exponential and reciprocal, each within a few ulp), summed in FP64:
// the molecular dynamics of FP32 handles.  The cutoff is the same exact
// integer test.
__device__ __forceinline__ void md_pair32(const uint4& ra, int qa, const uint4& rb, const MdPair& P, double f[3])
{
    const int32_t dx = (int32_t)(ra.x - rb.x), dy = (int32_t)(ra.y - rb.y), dz = (int32_t)(ra.z - rb.z);
    const uint32_t ax = (uint32_t)abs(dx), ay = (uint32_t)abs(dy), az = (uint32_t)abs(dz);
    const uint64_t r2i = (uint64_t)ax * ax + (uint64_t)ay * ay + (uint64_t)az * az;
    const float fx = (float)dx * P.sf, fy = (float)dy * P.sf, fz = (float)dz * P.sf;
    const float r2 = fx * fx + fy * fy + fz * fz;
    float g = 0.0f;
    const int qb = md_q(rb.w);
    if (r2i < P.R2 && qa != 0 && qb != 0) {
        const float rinv = __builtin_amdgcn_rsqf(r2), r = r2 * rinv;
        const float e = __builtin_amdgcn_exp2f(P.klf * r);
        g += P.lBf * (float)(qa * qb) * e * (1.0f + P.kappaf * r) * (rinv * rinv * rinv);
    }
    if (P.eps > 0.0 && r2 < 1.2599210498948731647672106f) {
        const float ir2 = __builtin_amdgcn_rcpf(r2), ir6 = ir2 * ir2 * ir2;
        g += 4.0f * P.epsf * (12.0f * ir6 * ir6 - 6.0f * ir6) * ir2;
    }
    f[0] += (double)(g * fx); f[1] += (double)(g * fy); f[2] += (double)(g * fz);
}

// the expanded excluded volume of core k on ion ra, added to f
__device__ __forceinline__ void md_core(const uint4& ra, const Replica& R, uint32_t k, const MdArgs& m, double s,
                                        double f[3])
{
    const uint4 cc = R.core_x[k];
    const int32_t dx = (int32_t)(ra.x - cc.x), dy = (int32_t)(ra.y - cc.y), dz = (int32_t)(ra.z - cc.z);
    const double fx = dx * s, fy = dy * s, fz = dz * s;
    const double r = sqrt(fx * fx + fy * fy + fz * fz);
    const double sh = r - R.core_delta[k];
    if (sh < 1.122462048309373) {
        const double ir = 1.0 / sh, ir2 = ir * ir, ir6 = ir2 * ir2 * ir2;
        const double g = 4.0 * m.eps * (12.0 * ir6 * ir6 - 6.0 * ir6) * ir / r;
        f[0] += g * fx; f[1] += g * fy; f[2] += g * fz;
    }
}

// one wavefront per cell of the replicas (global cell index from the
// flattened cell table), its lanes striding over the cell's slots
struct CellOf {
    uint32_t r, c, cnt;
    bool live;
};

__device__ __forceinline__ CellOf md_cell(const MdArgs& m, int buf)
{
    CellOf t{0u, 0u, 0u, false};
    const uint32_t gc = blockIdx.x;
    if (gc >= m.ncell_total) return t;
    t.r = m.cell2rep[gc];
    const Replica& R = m.reps[t.r];
    t.c = gc - R.cell_begin;
    t.cnt = R.cnt[buf][t.c];
    t.live = true;
    return t;
}

__global__ __launch_bounds__(64) void k_md_vinit(MdArgs m, int buf, uint64_t step)
{
    const CellOf t = md_cell(m, buf);
    if (!t.live) return;
    const Replica& R = m.reps[t.r];
    for (uint32_t j = threadIdx.x; j < t.cnt; j += blockDim.x) {
        const size_t slot = (size_t)t.c * R.cap + j;
        double v[3] = {0.0, 0.0, 0.0};
        if (md_is_ion(R.rec[buf][slot].w)) md_normals3(R, (uint32_t)step, t.c, j, TAG_MDVEL, v);
        double* vb = m.vel[t.r * 2 + buf] + 3 * slot;
        vb[0] = v[0]; vb[1] = v[1]; vb[2] = v[2];
    }
}

// Forces in the binning of buf; with langevin set, the drag and the noise of
// MD step `step` are added and the second half kick is applied.  One
// wavefront per cell: the records of the 27 cells around it (cells are at
// least rc wide) are staged in LDS once, segment by segment (the first
// MD_STAGE of them; the rest are read from memory).  The cell's ions, listed
// 64 slots at a time, each get a group of lanes (as many as fit all of them in
// one pass, a power of two) that split its partners, and each force is summed
// over its group.  (Screening the partners first and packing the interacting
// ones into a dense list was slower: the distance tests cost about as much as
// the pair terms they would skip.)
constexpr int MD_STAGE = 512;

// LDS written by one lane is read by others of the same wavefront in program
// order; this keeps the compiler from moving accesses across
__device__ __forceinline__ void md_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <bool F32>
__global__ __launch_bounds__(64) void k_md_force(MdArgs m, int buf, uint64_t step, int langevin)
{
    __shared__ uint4 nbr[MD_STAGE];
    const CellOf t = md_cell(m, buf);
    if (!t.live) return;
    const Replica& R = m.reps[t.r];
    const uint32_t lane = threadIdx.x, n = R.n, cap = R.cap, c = t.c;
    const uint32_t cx = c % n, cy = (c / n) % n, cz = c / (n * n);
    const uint4* recb = R.rec[buf];
    const uint32_t* cntb = R.cnt[buf];
    const double s = R.scale;
    const MdPair P{s, m.lB, R.kappa, m.eps, R.R2, (float)s, (float)m.lB, (float)R.kappa,
                   (float)(-R.kappa * 1.4426950408889634074), (float)m.eps};
    // lane o < 27: neighbour cell o (x fastest, offsets -1, 0, +1), its count
    // and where its records start in the concatenated list
    uint32_t ocell = 0u;
    int ocnt = 0;
    if (lane < 27) {
        const uint32_t x = (cx + n + (lane % 3) - 1u) % n, y = (cy + n + ((lane / 3) % 3) - 1u) % n,
                       z = (cz + n + (lane / 9) - 1u) % n;
        ocell = x + n * (y + n * z);
        ocnt = (int)cntb[ocell];
    }
    int pre = ocnt;
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) {
        const int v = __shfl_up(pre, off, 64);
        if ((int)lane >= off) pre += v;
    }
    const int ostart = pre - ocnt;
    const int total = __builtin_amdgcn_readlane(pre, 26);
    // the first 64 records of every segment, nine segments' loads in flight
    // at a time (each lane reads an in-range slot, the stores are masked),
    // then the rest of longer segments
    const auto seg_load = [&](int o) -> uint4 {
        const uint32_t oc = (uint32_t)__builtin_amdgcn_readlane((int)ocell, o);
        const int cn = __builtin_amdgcn_readlane(ocnt, o);
        return recb[(size_t)oc * cap + (uint32_t)min((int)lane, max(cn - 1, 0))];
    };
    const auto seg_store = [&](int o, const uint4& v) {
        const int cn = __builtin_amdgcn_readlane(ocnt, o), st = __builtin_amdgcn_readlane(ostart, o);
        if ((int)lane < cn && st + (int)lane < MD_STAGE) nbr[st + lane] = v;
    };
    for (int b = 0; b < 27; b += 9) {
        // nine loads, then nine stores (named registers, not an array the
        // compiler would place in scratch)
        const uint4 v0 = seg_load(b), v1 = seg_load(b + 1), v2 = seg_load(b + 2), v3 = seg_load(b + 3),
                    v4 = seg_load(b + 4), v5 = seg_load(b + 5), v6 = seg_load(b + 6), v7 = seg_load(b + 7),
                    v8 = seg_load(b + 8);
        seg_store(b, v0); seg_store(b + 1, v1); seg_store(b + 2, v2); seg_store(b + 3, v3); seg_store(b + 4, v4);
        seg_store(b + 5, v5); seg_store(b + 6, v6); seg_store(b + 7, v7); seg_store(b + 8, v8);
    }
    for (int o = 0; o < 27; ++o) {
        const uint32_t oc = (uint32_t)__builtin_amdgcn_readlane((int)ocell, o);
        const int cn = __builtin_amdgcn_readlane(ocnt, o), st = __builtin_amdgcn_readlane(ostart, o);
        for (int k = 64 + (int)lane; k < cn && st + k < MD_STAGE; k += 64) nbr[st + k] = recb[(size_t)oc * cap + k];
    }
    __syncthreads();
    __shared__ uint16_t ionj[64];
    const int self0 = __builtin_amdgcn_readlane(ostart, 13); // the centre cell's records in the list
    for (int b0 = 0; b0 < (int)t.cnt; b0 += 64) {
        // 64 slots at a time: their ions listed in slot order, the other
        // records (sites) get zero force
        const int jl = b0 + (int)lane;
        const bool have = jl < (int)t.cnt;
        const uint4 rj = have ? recb[(size_t)c * cap + jl] : make_uint4(0u, 0u, 0u, 0u);
        const bool is_ion = have && md_is_ion(rj.w);
        if (have && !is_ion) {
            double* fb = m.force[t.r] + 3 * ((size_t)c * cap + jl);
            fb[0] = fb[1] = fb[2] = 0.0;
        }
        const uint64_t im = __ballot(is_ion);
        const int nion = __popcll(im);
        if (is_ion) ionj[__popcll(im & ((1ull << lane) - 1ull))] = (uint16_t)(jl - b0);
        md_wave_sync();
        // lanes per ion: the largest power of two that fits them all in one pass
        int lg = 6;
        while (lg > 0 && (nion << lg) > 64) --lg;
        const int G = 1 << lg;
        const int gi = (int)lane >> lg, sub = (int)lane & (G - 1);
        for (int i0 = 0; i0 < nion; i0 += 64 >> lg) {
            const int i = i0 + gi;
            const bool act = i < nion;
            const int j = b0 + (int)ionj[act ? i : 0];
            const size_t slot = (size_t)c * cap + (size_t)j;
            const uint4 ra = recb[slot];
            double f[3] = {0.0, 0.0, 0.0};
            if (act && m.ion_coupling) { // ideal ions feel nothing
                const int qa = md_q(ra.w);
                // the staged part of the concatenated list in one stride
                const int self = self0 + j;
                for (int g = sub; g < min(total, MD_STAGE); g += G) {
                    if (g == self) continue;
                    if (F32) md_pair32(ra, qa, nbr[g], P, f);
                    else md_pair(ra, qa, nbr[g], P, f);
                }
                // the rest, segment by segment from memory
                if (total > MD_STAGE) {
                    for (int o = 0; o < 27; ++o) {
                        const uint32_t oc = (uint32_t)__builtin_amdgcn_readlane((int)ocell, o);
                        const int cn = __builtin_amdgcn_readlane(ocnt, o), st = __builtin_amdgcn_readlane(ostart, o);
                        for (int k = max(MD_STAGE - st, 0) + sub; k < cn; k += G) {
                            if (oc == c && k == j) continue;
                            if (F32) md_pair32(ra, qa, recb[(size_t)oc * cap + k], P, f);
                            else md_pair(ra, qa, recb[(size_t)oc * cap + k], P, f);
                        }
                    }
                }
                if (m.eps > 0.0)
                    for (uint32_t k = (uint32_t)sub; k < R.ncores; k += (uint32_t)G) md_core(ra, R, k, m, s, f);
            }
            for (int off = 1; off < G; off <<= 1) {
                f[0] += __shfl_xor(f[0], off, 64);
                f[1] += __shfl_xor(f[1], off, 64);
                f[2] += __shfl_xor(f[2], off, 64);
            }
            if (act && sub == 0) {
                if (langevin) {
                    double z[3];
                    md_normals3(R, (uint32_t)step, c, (uint32_t)j, TAG_MDNOISE, z);
                    double* vb = m.vel[t.r * 2 + buf] + 3 * slot;
                    for (int q = 0; q < 3; ++q) {
                        f[q] = f[q] - m.gamma * vb[q] + m.noise * z[q];
                        vb[q] += 0.5 * m.dt * f[q];
                    }
                }
                double* fb = m.force[t.r] + 3 * slot;
                fb[0] = f[0]; fb[1] = f[1]; fb[2] = f[2];
            }
        }
        md_wave_sync(); // the ion list is rewritten for the next slots
    }
}

__global__ __launch_bounds__(64) void k_md_drift(MdArgs m, int buf)
{
    const CellOf t = md_cell(m, buf);
    if (!t.live) return;
    const Replica& R = m.reps[t.r];
    const double to_lat = 4294967296.0 / R.L;
    for (uint32_t j = threadIdx.x; j < t.cnt; j += blockDim.x) {
        const size_t slot = (size_t)t.c * R.cap + j;
        uint4& ra = R.rec[buf][slot];
        if (!md_is_ion(ra.w)) continue;
        double* vb = m.vel[t.r * 2 + buf] + 3 * slot;
        const double* fb = m.force[t.r] + 3 * slot;
        uint32_t x[3] = {ra.x, ra.y, ra.z};
        for (int q = 0; q < 3; ++q) {
            vb[q] += 0.5 * m.dt * fb[q];
            x[q] = (uint32_t)((long long)x[q] + llround(m.dt * vb[q] * to_lat));
        }
        ra.x = x[0]; ra.y = x[1]; ra.z = x[2];
    }
}

// the records (and velocities) of buf re-binned into buf ^ 1 in the same grid
__global__ __launch_bounds__(64) void k_md_rebin(MdArgs m, int buf)
{
    const uint32_t gc = blockIdx.x;
    if (gc >= m.ncell_total) return;
    const uint32_t r = m.cell2rep[gc];
    const Replica& R = m.reps[r];
    const uint32_t c = gc - R.cell_begin, n = R.n, cap = R.cap;
    const uint32_t cx = c % n, cy = (c / n) % n, cz = c / (n * n);
    const uint32_t lane = threadIdx.x;
    const uint32_t o0 = R.tab->o[0], o1 = R.tab->o[1], o2 = R.tab->o[2];
    // the 27 cells around c, their counts loaded at once
    uint32_t nb = 0xFFFFFFFFu, ncnt = 0u;
    if (lane < 27) {
        const uint32_t x = (cx + n + (lane % 3) - 1u) % n, y = (cy + n + ((lane / 3) % 3) - 1u) % n,
                       z = (cz + n + (lane / 9) - 1u) % n;
        nb = x + n * (y + n * z);
        ncnt = R.cnt[buf][nb];
    }
    // rank of this lane's cell among the 27 (distinct when n >= 3)
    uint32_t rank = 0;
    for (int q = 0; q < 27; ++q) {
        const uint32_t v = (uint32_t)__shfl((int)nb, q, 64);
        rank += (v < nb) ? 1u : 0u;
    }
    const uint4* src = R.rec[buf];
    const double* vsrc = m.vel[r * 2 + buf];
    uint4* dst = R.rec[buf ^ 1];
    double* vdst = m.vel[r * 2 + (buf ^ 1)];
    // lane q < 27: the source cell of rank q and its count (ascending index)
    const uint32_t to = lane < 27 ? rank : lane;
    const uint32_t qcell = (uint32_t)__builtin_amdgcn_ds_permute((int)(to << 2), (int)nb);
    const uint32_t qcnt = (uint32_t)__builtin_amdgcn_ds_permute((int)(to << 2), (int)ncnt);
    uint32_t out = 0;
    // a slot's record goes to this cell if it falls into it: appended in order
    const auto take = [&](uint32_t sc, uint32_t k, bool valid, const uint4& rec) {
        bool mine = false;
        if (valid) {
            const uint32_t nx = __umulhi(rec.x - o0, n), ny = __umulhi(rec.y - o1, n), nz = __umulhi(rec.z - o2, n);
            mine = nx + n * (ny + n * nz) == c;
        }
        const uint64_t mask = __ballot(mine);
        const uint32_t before = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
        if (mine) {
            const uint32_t at = out + before;
            if (at < cap) {
                dst[(size_t)c * cap + at] = rec;
                const double* vs = vsrc + 3 * ((size_t)sc * cap + k);
                double* vd = vdst + 3 * ((size_t)c * cap + at);
                vd[0] = vs[0]; vd[1] = vs[1]; vd[2] = vs[2];
            }
        }
        out += (uint32_t)__popcll(mask);
    };
    // the first 64 records of nine source cells in flight at a time (each lane
    // reads an in-range slot), taken in rank order, longer cells finished
    // before the next rank
    for (int b = 0; b < 27; b += 9) {
        uint4 v[9];
#pragma unroll
        for (int u = 0; u < 9; ++u) {
            const uint32_t sc = (uint32_t)__builtin_amdgcn_readlane((int)qcell, b + u);
            const uint32_t cn = (uint32_t)__builtin_amdgcn_readlane((int)qcnt, b + u);
            v[u] = src[(size_t)sc * cap + (cn ? min(lane, cn - 1u) : 0u)];
        }
        for (int u = 0; u < 9; ++u) {
            const uint32_t sc = (uint32_t)__builtin_amdgcn_readlane((int)qcell, b + u);
            const uint32_t cn = (uint32_t)__builtin_amdgcn_readlane((int)qcnt, b + u);
            take(sc, lane, lane < cn, v[u]);
            for (uint32_t b0 = 64; b0 < cn; b0 += 64) {
                const uint32_t k = b0 + lane;
                take(sc, k, k < cn, k < cn ? src[(size_t)sc * cap + k] : make_uint4(0u, 0u, 0u, 0u));
            }
        }
    }
    if (lane == 0) {
        R.cnt[buf ^ 1][c] = out < cap ? out : cap;
        if (out > cap) atomicOr(m.err, ERR_BIN_CAPACITY);
        atomicMax(R.hiwater, out);
    }
}

hipError_t launch_md_block(const MdArgs& m, int buf0, uint64_t step0, int64_t nsteps, uint32_t maxcap, hipStream_t s,
                           int* buf_out)
{
    (void)maxcap;
    const dim3 grid(m.ncell_total), block(64);
    int buf = buf0;
    hipLaunchKernelGGL(k_md_vinit, grid, block, 0, s, m, buf, step0);
    const auto force = m.precision == 32 ? k_md_force<true> : k_md_force<false>;
    hipLaunchKernelGGL(force, grid, block, 0, s, m, buf, step0, 0);
    for (int64_t st = 0; st < nsteps; ++st) {
        hipLaunchKernelGGL(k_md_drift, grid, block, 0, s, m, buf);
        hipLaunchKernelGGL(k_md_rebin, dim3(m.ncell_total), dim3(64), 0, s, m, buf);
        buf ^= 1;
        hipLaunchKernelGGL(force, grid, block, 0, s, m, buf, step0 + (uint64_t)st, 1);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    *buf_out = buf;
    return hipGetLastError();
}

} // namespace crmc

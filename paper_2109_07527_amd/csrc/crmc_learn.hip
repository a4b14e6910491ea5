// CDNA4 (gfx950) kernels of the learned site proposal.
//
//   k_learn<R>   per colour phase: for the sites of every active cell, the
//                environment features (charged particles of the 26 neighbour
//                cells within rc, by radial shell and sign relative to the
//                site's ionized charge); a labelled training row per site
//                while rows are being collected; with the proposal on, the
//                network output p = logistic of a 32 -> 128 -> 128 -> 1 ReLU
//                perceptron.  R = float: BF16 matrix cores
//                (v_mfma_f32_16x16x32_bf16) with FP32 accumulation;
//                R = double: FP64, vector unit.
//   k_mlp_grad   mean binary cross-entropy gradient of a minibatch on the
//                matrix cores (BF16 operands, FP32 accumulation; 16x16x32
//                products, and 16x16x16 for the weight gradients, whose K is
//                the wavefront's 16 rows).
//   k_adam       Adam step on the FP32 master parameters, refreshing the
//                BF16 copies the inference uses.
//   k_mlp_fwd    logits of given feature rows (the same network code as k_learn<float>).
//
// The neighbour cells are inactive during the phase, so the outputs fix the
// proposal weights of the phase's trials (detailed balance holds for the
// frozen environment).
#include "crmc_internal.h"

namespace crmc {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// gfx950's 16x16x32 BF16 matrix product (FP32 accumulate): lane (col, grp)
// supplies A[col][8 grp + e] and B[8 grp + e][col], e = 0..7, and receives
// D[4 grp + e][col], e = 0..3.  Any pairing of the K indices that A and B
// share gives the same product, so only that they share it matters.
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c,
                                                   0, 0, 0);
}

constexpr int LIN = MLP_IN, LH = MLP_H;
static_assert(LIN % 32 == 0 && LH % 32 == 0, "the products step K by 32");
constexpr int SITES_PER_WG = 64;    // sites of one cell handled by one workgroup
constexpr int LEARN_THREADS = 512;  // eight wavefronts: each takes every 8th kept record
constexpr int LEARN_WAVES = LEARN_THREADS / 64;
constexpr int RAW_PER_THREAD = 6;
constexpr int STAGE = LEARN_THREADS * RAW_PER_THREAD; // neighbour records examined per round

__device__ __forceinline__ uint64_t lanes_below()
{
    const uint32_t lane = threadIdx.x & 63u;
    return lane ? (~0ull >> (64u - lane)) : 0ull;
}

// round-to-nearest-even float -> bf16 bits
__device__ __forceinline__ short f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}

__device__ __forceinline__ int q_of(uint32_t meta)
{
    const uint32_t k = meta & 7u, c = (meta >> 3) & 1u;
    if (k == KIND_ACID) return -(int)c;
    if (k == KIND_BASE) return (int)c;
    if (k == KIND_XPOS) return 1;
    if (k == KIND_XNEG) return -1;
    return 0;
}

// ---------------------------------------------------------------------------
// the network on 16 rows per wavefront (BF16 matrix cores, FP32 accumulate)
// ---------------------------------------------------------------------------
// LDS operands: W1b [128][32] and W2b [128][128] as bf16 (row = output
// unit); X [16][32] bf16 rows of this wavefront; H [16][128] bf16 scratch.
// Rows are XS, HS, W1S, W2S elements apart (padding spreads the 16 rows a
// matrix-core operand reads across the LDS banks).  Returns the logit of
// row (lane & 15) in every lane of that row group.
template <int XS = MLP_IN, int HS = MLP_H, int W1S = MLP_IN, int W2S = MLP_H>
__device__ __forceinline__ float mlp_rows16(const short* W1b, const short* W2b, const float* b1, const float* b2,
                                            const float* w3, float b3, const short* X, short* H, float* h2out)
{
    const int l = threadIdx.x & 63;
    const int col = l & 15, grp = l >> 4;
    // layer 1: D[m][n] = sum_k X[m][k] W1[n][k]
    f32x4 acc[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < LIN / 32; ++ks) {
        bf16x8 a;
#pragma unroll
        for (int e = 0; e < 8; ++e) a[e] = X[col * XS + ks * 32 + 8 * grp + e];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            bf16x8 b;
#pragma unroll
            for (int e = 0; e < 8; ++e) b[e] = W1b[(t * 16 + col) * W1S + ks * 32 + 8 * grp + e];
            acc[t] = mfma32(a, b, acc[t]);
        }
    }
    // bias, ReLU, to LDS as bf16 (row-major [m][n])
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int m = 4 * grp + e, n = t * 16 + col;
            const float v = acc[t][e] + b1[n];
            H[m * HS + n] = f2bf(v > 0.f ? v : 0.f);
        }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // layer 2: D[m][n] = sum_k H1[m][k] W2[n][k]
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int ks = 0; ks < LH / 32; ++ks) {
        bf16x8 a;
#pragma unroll
        for (int e = 0; e < 8; ++e) a[e] = H[col * HS + ks * 32 + 8 * grp + e];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            bf16x8 b;
#pragma unroll
            for (int e = 0; e < 8; ++e) b[e] = W2b[(t * 16 + col) * W2S + ks * 32 + 8 * grp + e];
            acc[t] = mfma32(a, b, acc[t]);
        }
    }
    // bias, ReLU, dot with w3: lane (col, grp) sums its 8 columns for rows 4 grp + e
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int n = t * 16 + col;
            float v = acc[t][e] + b2[n];
            v = v > 0.f ? v : 0.f;
            if (h2out) h2out[(4 * grp + e) * LH + n] = v;
            part[e] += v * w3[n];
        }
    // sum over the 16 columns of a row group (lanes grp*16 .. grp*16+15)
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) part[e] += __shfl_xor(part[e], off, 16);
    // logit of row (lane & 15): held by group (row / 4), element row % 4
    const int row = l & 15;
    const float z0 = __shfl(part[0], (row >> 2) * 16, 64), z1 = __shfl(part[1], (row >> 2) * 16, 64);
    const float z2 = __shfl(part[2], (row >> 2) * 16, 64), z3 = __shfl(part[3], (row >> 2) * 16, 64);
    const int e = row & 3;
    return (e == 0 ? z0 : e == 1 ? z1 : e == 2 ? z2 : z3) + b3;
}

// FP64 network on one feature row (vector unit)
__device__ double mlp_row_f64(const double* P, const double* x)
{
    double h1[LH];
    for (int o = 0; o < LH; ++o) {
        double a = P[MLP_B1 + o];
        for (int i = 0; i < LIN; ++i) a += P[o * LIN + i] * x[i];
        h1[o] = a > 0.0 ? a : 0.0;
    }
    double z = P[MLP_B3];
    for (int o = 0; o < LH; ++o) {
        double a = P[MLP_B2 + o];
        for (int i = 0; i < LH; ++i) a += P[MLP_W2 + o * LH + i] * h1[i];
        if (a > 0.0) z += P[MLP_W3 + o] * a;
    }
    return z;
}

__device__ __forceinline__ double site_prob(double z)
{
    double p = 1.0 / (1.0 + exp(-z));
    return p < 1e-6 ? 1e-6 : (p > 1.0 - 1e-6 ? 1.0 - 1e-6 : p);
}

// ---------------------------------------------------------------------------
// k_learn: features and network outputs of the sites of a phase
// ---------------------------------------------------------------------------
// Work item (replica, cell, part): the cell's sites of rank 64 part ..
// 64 part + 63 in its record order (no kernel moves records during this
// launch), counted against the charged records of the 26 neighbour cells by
// one workgroup, which then writes the training rows while rows are being
// collected and, with the proposal on, evaluates the network on the item's
// rows (R = float: BF16 matrix cores with the weights held in LDS for all its
// items; R = double: FP64 per thread).  The workgroups stride over the
// phase's items.  The loads of an item are issued in as few dependent rounds
// as possible (item, then the cell counts, then the own and neighbour records
// together): the kernel is bound by memory latency, not by arithmetic.
constexpr int XS = LIN + 8, HS = LH + 8, W1S = LIN + 8, W2S = LH + 8; // padded LDS rows

struct LearnShared {
    uint4 site[SITES_PER_WG];             // x, y, z, meta of the item's sites
    int hist[SITES_PER_WG][LIN + 1];      // counts (rows padded against bank conflicts)
    int seg[27];                          // prefix of the 26 neighbour counts
    uint32_t segcell[26];
    int box[6];                           // least and largest site offsets from site 0 per axis
    int wcount[LEARN_WAVES];
    int kcount[RAW_PER_THREAD][LEARN_WAVES]; // kept records per round slot and wavefront
    uint64_t r2sh[17];
};

// dynamic LDS: kept neighbour records, then (FP32 network) the padded BF16
// weights, the per-wave X and H tiles, and b1, b2, w3, b3
size_t learn_stage_bytes() { return sizeof(int4) * STAGE; }
size_t learn_infer_lds_bytes()
{
    return learn_stage_bytes() + sizeof(short) * (LH * W1S + LH * W2S + 4 * 16 * XS + 4 * 16 * HS) +
           sizeof(float) * (3 * LH + 4);
}

__device__ __forceinline__ int wave_min(int v)
{
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ int wave_max(int v)
{
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

template <typename Real>
__global__ __launch_bounds__(LEARN_THREADS) void k_learn(SweepArgs a, LearnArgs g)
{
    __shared__ LearnShared S;
    extern __shared__ uint4 lsh4[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int colour = a.colour;
    const uint32_t nwork = min(a.plan_n[plan_idx(colour, PLAN_LWORK)], a.lwork_cap);
    if (blockIdx.x >= nwork) return;
    const uint64_t s = *a.sweep;
    const int buf = (int)((s + 1u) & 1u);
    const bool mfma = sizeof(Real) == 4 && g.infer;
    int4* nb = (int4*)lsh4; // kept records: offsets from site 0, 16 for a positive charge else 0
    short* W1b = (short*)(lsh4 + STAGE);
    short* W2b = W1b + LH * W1S;
    short* Xw = W2b + LH * W2S + (wave & 3) * (16 * XS);
    short* Hw = W2b + LH * W2S + 4 * 16 * XS + (wave & 3) * (16 * HS);
    float* b1 = (float*)(W2b + LH * W2S + 4 * 16 * XS + 4 * 16 * HS);
    float* b2 = b1 + LH;
    float* w3 = b2 + LH;
    if (mfma) {
        // padded copies of the BF16 weights (rows of 16-byte chunks) and the FP32 vectors
        const uint4* gw1 = (const uint4*)g.w1b;
        const uint4* gw2 = (const uint4*)g.w2b;
        for (int i = tid; i < LH * LIN / 8; i += LEARN_THREADS)
            *(uint4*)(W1b + (i / (LIN / 8)) * W1S + (i % (LIN / 8)) * 8) = gw1[i];
        for (int i = tid; i < LH * LH / 8; i += LEARN_THREADS)
            *(uint4*)(W2b + (i / (LH / 8)) * W2S + (i % (LH / 8)) * 8) = gw2[i];
        if (tid <= 3 * LH) // b1, b2, then w3 and b3 (stored after w3)
            b1[tid] = g.p32[tid < LH ? MLP_B1 + tid : (tid < 2 * LH ? MLP_B2 + tid - LH : MLP_W3 + tid - 2 * LH)];
    }
    for (uint32_t it = blockIdx.x; it < nwork; it += gridDim.x) {
        const LearnItem& I = a.lwork[(size_t)colour * a.lwork_cap + it];
        const uint32_t r = I.r, cell = I.cell, part = I.part, n = I.n, cap = I.cap;
        const uint4* recb = I.rec;
        const uint32_t* cntb = I.cnt;
        double* phat = I.phat;
        const double off_acid = I.off[0], off_base = I.off[1];
        const int lo = (int)part * SITES_PER_WG;
        // the cell's records are read before its count arrives (the slots up
        // to the capacity are all inside the cell's storage)
        uint4 own = make_uint4(0, 0, 0, 0);
        if (tid < (int)cap) own = recb[(size_t)cell * cap + tid];
        const int nown = (int)cntb[cell];

        // neighbour cells and the prefix of their counts (wave 0), thresholds, cleared counts
        if (wave == 0) {
            int cv = 0;
            if (lane < 26) {
                const uint32_t cx = cell % n, cy = (cell / n) % n, cz = cell / (n * n);
                const int oo = lane < 13 ? lane : lane + 1;
                const uint32_t x = (cx + n + (uint32_t)(oo % 3) - 1u) % n,
                               y = (cy + n + (uint32_t)((oo / 3) % 3) - 1u) % n, z = (cz + n + (uint32_t)(oo / 9) - 1u) % n;
                const uint32_t c = x + n * (y + n * z);
                S.segcell[lane] = c;
                cv = (int)cntb[c];
            }
            for (int off = 1; off < 32; off <<= 1) {
                const int y = __shfl_up(cv, off, 64);
                if (lane >= off) cv += y;
            }
            if (lane < 26) S.seg[lane + 1] = cv;
            if (lane == 0) S.seg[0] = 0;
        }
        if (tid >= 64 && tid < 64 + 17) S.r2sh[tid - 64] = g.R2sh[(size_t)r * 17 + tid - 64];
        for (int i = tid; i < SITES_PER_WG * (LIN + 1); i += LEARN_THREADS) (&S.hist[0][0])[i] = 0;
        __syncthreads();
        const int nbt = S.seg[26];

        // the first round of neighbour records, in flight while the sites are ranked
        uint4 v[RAW_PER_THREAD];
        const int rr1 = min(nbt, STAGE);
#pragma unroll
        for (int u = 0; u < RAW_PER_THREAD; ++u) {
            const int i = u * LEARN_THREADS + tid;
            v[u] = make_uint4(0, 0, 0, 0);
            if (i < rr1) {
                int q = 0, hi = 26; // seg[q] <= i < seg[hi]
                while (hi - q > 1) {
                    const int mid = (q + hi) >> 1;
                    if (S.seg[mid] <= i) q = mid; else hi = mid;
                }
                v[u] = recb[(size_t)S.segcell[q] * cap + (uint32_t)(i - S.seg[q])];
            }
        }

        // the item's sites: rank among the cell's sites (block prefix over wave ballots)
        int base = 0;
        for (int b0 = 0; b0 < nown; b0 += LEARN_THREADS) {
            const int i = b0 + tid;
            uint4 o = make_uint4(0, 0, 0, 0);
            bool site = false;
            if (i < nown) {
                o = b0 == 0 ? own : recb[(size_t)cell * cap + i];
                const uint32_t k = o.w & 7u;
                site = k == KIND_ACID || k == KIND_BASE;
            }
            const uint64_t mask = __ballot(site);
            if (lane == 0) S.wcount[wave] = __popcll(mask);
            __syncthreads();
            int before = base, tot = 0;
            for (int q = 0; q < LEARN_WAVES; ++q) {
                before += q < wave ? S.wcount[q] : 0;
                tot += S.wcount[q];
            }
            const int rank = before + __popcll(mask & lanes_below());
            if (site && rank >= lo && rank < lo + SITES_PER_WG) S.site[rank - lo] = o;
            base += tot;
            __syncthreads();
        }
        const int nsite = base <= lo ? 0 : min(SITES_PER_WG, base - lo);
        if (nsite == 0) continue; // uniform: base is the same in every thread

        const uint4 s0 = S.site[0];
        int so[3] = {0, 0, 0}; // this lane's site as offsets from site 0
        int sq = 0;            // 16 when the site's ionized charge is positive
        if (lane < nsite) {
            const uint4 me = S.site[lane];
            so[0] = (int32_t)(me.x - s0.x);
            so[1] = (int32_t)(me.y - s0.y);
            so[2] = (int32_t)(me.z - s0.z);
            sq = (me.w & 7u) == KIND_ACID ? 0 : 16;
        }
        if (wave == 0) {
            // the sites' bounding box (offsets from site 0; absent lanes repeat site 0)
            for (int d = 0; d < 3; ++d) {
                const int mn = wave_min(so[d]), mx = wave_max(so[d]);
                if (lane == 0) {
                    S.box[d] = mn;
                    S.box[3 + d] = mx;
                }
            }
        }
        __syncthreads();
        const uint64_t* R2sh = S.r2sh;
        const uint64_t R2 = R2sh[16];
        // Shell k holds sqrt(d2) / c in [k, k + 1) with c = rc / 16 in lattice
        // units.  The float offsets are within 2^-24 relative of the exact ones,
        // so the float quotient t is off by far less than 1e-4: it decides
        // unless it lies within 1e-4 of an integer up to 16, where the integer
        // thresholds do.
        const float inv_c = 16.0f / sqrtf((float)R2);
        // a record at a squared distance of R2 or more from the sites' bounding
        // box is at least that far from every site and cannot count
        const int blo[3] = {S.box[0], S.box[1], S.box[2]};
        const int bhi[3] = {S.box[3], S.box[4], S.box[5]};
        const float sfx = (float)so[0], sfy = (float)so[1], sfz = (float)so[2];
        const int hrow = lane * (LIN + 1) + 16; // - (code ^ sq) + k: channel 16 for equal signs, else 0

        for (int r0 = 0; r0 < nbt; r0 += STAGE) {
            const int r1 = min(nbt, r0 + STAGE);
            if (r0 > 0) {
                // a further round (more than STAGE neighbour records)
                __syncthreads();
#pragma unroll
                for (int u = 0; u < RAW_PER_THREAD; ++u) {
                    const int i = r0 + u * LEARN_THREADS + tid;
                    v[u] = make_uint4(0, 0, 0, 0);
                    if (i < r1) {
                        int q = 0, hi = 26;
                        while (hi - q > 1) {
                            const int mid = (q + hi) >> 1;
                            if (S.seg[mid] <= i) q = mid; else hi = mid;
                        }
                        v[u] = recb[(size_t)S.segcell[q] * cap + (uint32_t)(i - S.seg[q])];
                    }
                }
                __syncthreads();
            }
            // keep the charged records near the sites, compacted in (slot, wavefront) order
            uint64_t km[RAW_PER_THREAD];
            int kx[RAW_PER_THREAD], ky[RAW_PER_THREAD], kz[RAW_PER_THREAD], kq[RAW_PER_THREAD];
#pragma unroll
            for (int u = 0; u < RAW_PER_THREAD; ++u) {
                const int i = r0 + u * LEARN_THREADS + tid;
                const int qq = i < r1 ? q_of(v[u].w) : 0;
                kx[u] = (int32_t)(v[u].x - s0.x);
                ky[u] = (int32_t)(v[u].y - s0.y);
                kz[u] = (int32_t)(v[u].z - s0.z);
                kq[u] = qq > 0 ? 16 : 0;
                const int64_t x = kx[u], y = ky[u], z = kz[u];
                // gaps clamped at 2^31 (R2 < 2^60 since rc <= L / 4), so the sum cannot wrap
                const int64_t cl = (int64_t)1 << 31;
                const uint64_t ex = (uint64_t)min(max(max((int64_t)blo[0] - x, x - (int64_t)bhi[0]), (int64_t)0), cl);
                const uint64_t ey = (uint64_t)min(max(max((int64_t)blo[1] - y, y - (int64_t)bhi[1]), (int64_t)0), cl);
                const uint64_t ez = (uint64_t)min(max(max((int64_t)blo[2] - z, z - (int64_t)bhi[2]), (int64_t)0), cl);
                const bool keep = qq != 0 && ex * ex + ey * ey + ez * ez < R2;
                km[u] = __ballot(keep);
                if (lane == 0) S.kcount[u][wave] = __popcll(km[u]);
            }
            __syncthreads();
            int ns = 0;
#pragma unroll
            for (int u = 0; u < RAW_PER_THREAD; ++u) {
                int before = ns;
                for (int q = 0; q < LEARN_WAVES; ++q) {
                    before += q < wave ? S.kcount[u][q] : 0;
                    ns += S.kcount[u][q];
                }
                if ((km[u] >> lane) & 1ull)
                    nb[before + __popcll(km[u] & lanes_below())] = make_int4(kx[u], ky[u], kz[u], kq[u]);
            }
            __syncthreads();
            if (lane < nsite) {
                for (int j = wave; j < ns; j += LEARN_WAVES) {
                    const int4 o = nb[j];
                    const float dx = (float)o.x - sfx, dy = (float)o.y - sfy, dz = (float)o.z - sfz;
                    const float d2f = dx * dx + dy * dy + dz * dz;
                    const float t = __builtin_amdgcn_sqrtf(d2f) * inv_c;
                    const float tr = __builtin_rintf(t);
                    bool inr = t < 16.0f;
                    int k = (int)t;
                    if (fabsf(t - tr) < 1e-4f && tr < 16.5f) {
                        // near a shell boundary or the cutoff: the exact integer thresholds
                        const uint32_t ax = (uint32_t)abs((int32_t)((uint32_t)o.x - (uint32_t)so[0]));
                        const uint32_t ay = (uint32_t)abs((int32_t)((uint32_t)o.y - (uint32_t)so[1]));
                        const uint32_t az = (uint32_t)abs((int32_t)((uint32_t)o.z - (uint32_t)so[2]));
                        const uint64_t d2 = (uint64_t)ax * ax + (uint64_t)ay * ay + (uint64_t)az * az;
                        inr = d2 < R2;
                        k = k > 15 ? 15 : k;
                        while (k > 0 && d2 < R2sh[k]) --k;
                        while (k < 15 && d2 >= R2sh[k + 1]) ++k;
                    }
                    if (inr) atomicAdd(&(&S.hist[0][0])[hrow - (o.w ^ sq) + k], 1);
                }
            }
            __syncthreads();
        }

        // recorded features (checks): per site, as evaluated in this phase
        if (I.feat && tid < nsite) {
            float* f = I.feat + (size_t)(S.site[tid].w >> 8) * LIN;
            for (int i = 0; i < LIN; ++i) f[i] = (float)S.hist[tid][i];
        }
        // training rows: the features and the site's ionization at the start of the phase
        if (g.data && tid < nsite) {
            const unsigned long long row = atomicAdd(g.data_n, 1ull);
            if (row < g.data_cap) {
                for (int i = 0; i < LIN; ++i) g.data[row * (LIN + 1) + i] = (float)S.hist[tid][i];
                g.data[row * (LIN + 1) + LIN] = (float)((S.site[tid].w >> 3) & 1u);
            }
        }
        if (g.infer) {
            if (mfma) {
                const int row0 = wave * 16;
                if (row0 < nsite) {
                    for (int i = lane; i < 16 * LIN; i += 64) {
                        const int rr = row0 + i / LIN;
                        Xw[(i / LIN) * XS + i % LIN] = rr < nsite ? f2bf((float)S.hist[rr][i % LIN]) : (short)0;
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    const float z = mlp_rows16<XS, HS, W1S, W2S>(W1b, W2b, b1, b2, w3, w3[LH], Xw, Hw, nullptr);
                    const int rr = row0 + (lane & 15);
                    if (lane < 16 && rr < nsite) {
                        const uint32_t m = S.site[rr].w;
                        phat[m >> 8] = site_prob((double)z + ((m & 7u) == KIND_ACID ? off_acid : off_base));
                    }
                }
            } else if (tid < nsite) {
                double x[LIN];
                for (int i = 0; i < LIN; ++i) x[i] = (double)S.hist[tid][i];
                const uint32_t m = S.site[tid].w;
                phat[m >> 8] = site_prob(mlp_row_f64(g.p64, x) + ((m & 7u) == KIND_ACID ? off_acid : off_base));
            }
        }
        __syncthreads();
    }
}

// logits of given rows (tests): 64 rows per workgroup
__global__ __launch_bounds__(256) void k_mlp_fwd(LearnArgs g, const float* X, int nrows, float* out)
{
    extern __shared__ short lsh[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    short* W1b = lsh;
    short* W2b = W1b + LH * LIN;
    short* Xw = W2b + LH * LH + wave * (16 * LIN);
    short* Hw = W2b + LH * LH + 4 * 16 * LIN + wave * (16 * LH);
    for (int i = tid; i < LH * LIN; i += 256) W1b[i] = g.w1b[i];
    for (int i = tid; i < LH * LH; i += 256) W2b[i] = g.w2b[i];
    __syncthreads();
    const int row0 = blockIdx.x * 64 + wave * 16;
    for (int i = lane; i < 16 * LIN; i += 64) {
        const int rr = row0 + i / LIN;
        Xw[i] = rr < nrows ? f2bf(X[(size_t)rr * LIN + i % LIN]) : (short)0;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const float z = mlp_rows16(W1b, W2b, g.p32 + MLP_B1, g.p32 + MLP_B2, g.p32 + MLP_W3, g.p32[MLP_B3], Xw, Hw, nullptr);
    const int rr = row0 + (lane & 15);
    if (lane < 16 && rr < nrows) out[rr] = z;
}

// ---------------------------------------------------------------------------
// k_mlp_grad: minibatch gradient (rows of data: 32 features + label)
// ---------------------------------------------------------------------------
// Each wavefront takes 16 rows; the workgroup's weight gradients are added
// to grad (FP32) with atomics; loss (FP64) likewise.  Operands of every
// product are BF16, accumulation FP32.
__global__ __launch_bounds__(256) void k_mlp_grad(LearnArgs g, const float* data, const int* rows, int nrows,
                                                  float inv_batch, float* grad, double* loss)
{
    extern __shared__ short lsh[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int col = lane & 15, grp = lane >> 4;
    short* W1b = lsh;                                   // [128][32]
    short* W2b = W1b + LH * LIN;                        // [128][128]
    short* Xw = W2b + LH * LH + wave * (16 * LIN);      // [16][32]  rows x features
    short* Hw = W2b + LH * LH + 4 * 16 * LIN + wave * (16 * LH); // [16][128] H1 (bf16)
    float* fbase = reinterpret_cast<float*>(W2b + LH * LH + 4 * 16 * LIN + 4 * 16 * LH);
    float* H2 = fbase + wave * (16 * LH);               // [16][128] H2 (fp32, after ReLU)
    float* D2 = fbase + 4 * 16 * LH + wave * (16 * LH); // [16][128] dA2, then dA1 (fp32)
    short* D2b = reinterpret_cast<short*>(fbase + 8 * 16 * LH) + wave * (16 * LH); // bf16 copy
    for (int i = tid; i < LH * LIN; i += 256) W1b[i] = g.w1b[i];
    for (int i = tid; i < LH * LH; i += 256) W2b[i] = g.w2b[i];
    __syncthreads();
    const int row0 = blockIdx.x * 64 + wave * 16;
    float yv = 0.f;
    for (int i = lane; i < 16 * LIN; i += 64) {
        const int rr = row0 + i / LIN;
        Xw[i] = rr < nrows ? f2bf(data[(size_t)rows[rr] * (LIN + 1) + i % LIN]) : (short)0;
    }
    if (lane < 16 && row0 + lane < nrows) yv = data[(size_t)rows[row0 + lane] * (LIN + 1) + LIN];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const float* b1 = g.p32 + MLP_B1;
    const float* b2 = g.p32 + MLP_B2;
    const float* w3 = g.p32 + MLP_W3;
    const float z = mlp_rows16(W1b, W2b, b1, b2, w3, g.p32[MLP_B3], Xw, Hw, H2);
    // per row (lane < 16): dz = (sigmoid(z) - y) / B, loss
    const bool live = lane < 16 && row0 + lane < nrows;
    float dz = 0.f;
    if (live) {
        dz = (1.f / (1.f + __expf(-z)) - yv) * inv_batch;
        const double zd = z;
        const double l = (zd > 0.0 ? zd + log1p(exp(-zd)) : log1p(exp(zd))) - (double)yv * zd;
        atomicAdd(loss, l * (double)inv_batch);
    }
    // dw3[n] = sum_m dz_m H2[m][n]; db3; dA2[m][n] = dz_m w3[n] [H2 > 0]
    for (int nn = lane; nn < LH; nn += 64) {
        float s = 0.f;
        for (int mm = 0; mm < 16; ++mm) s += __shfl(dz, mm, 64) * H2[mm * LH + nn];
        atomicAdd(&grad[MLP_W3 + nn], s);
    }
    {
        float sdz = lane < 16 ? dz : 0.f;
        for (int off = 8; off > 0; off >>= 1) sdz += __shfl_xor(sdz, off, 64);
        if (lane == 0) atomicAdd(&grad[MLP_B3], sdz);
    }
    for (int i = lane; i < 16 * LH; i += 64) {
        const int mm = i / LH, nn = i % LH;
        const float dzm = __shfl(dz, mm, 64); // every lane takes part in the exchange
        const float v = H2[i] > 0.f ? dzm * w3[nn] : 0.f;
        D2[i] = v;
        D2b[i] = f2bf(v);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // db2[n] = sum_m dA2[m][n]
    for (int nn = lane; nn < LH; nn += 64) {
        float s = 0.f;
        for (int mm = 0; mm < 16; ++mm) s += D2[mm * LH + nn];
        atomicAdd(&grad[MLP_B2 + nn], s);
    }
    // dW2[o][i] = sum_m dA2[m][o] H1[m][i]: A = dA2^T (M = o, K = m), B = H1 (K = m, N = i)
    for (int to = 0; to < 8; ++to) {
        bf16x4 av;
#pragma unroll
        for (int e = 0; e < 4; ++e) av[e] = D2b[(4 * grp + e) * LH + to * 16 + col];
#pragma unroll
        for (int ti = 0; ti < 8; ++ti) {
            bf16x4 bv;
#pragma unroll
            for (int e = 0; e < 4; ++e) bv[e] = Hw[(4 * grp + e) * LH + ti * 16 + col];
            f32x4 c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; ++e)
                atomicAdd(&grad[MLP_W2 + (to * 16 + 4 * grp + e) * LH + ti * 16 + col], c[e]);
        }
    }
    // dH1[m][i] = sum_o dA2[m][o] W2[o][i]: A = dA2 (M = m, K = o), B = W2 (K = o, N = i)
    f32x4 dh[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) dh[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < LH / 32; ++ks) {
        bf16x8 av;
#pragma unroll
        for (int e = 0; e < 8; ++e) av[e] = D2b[col * LH + ks * 32 + 8 * grp + e];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            bf16x8 bv;
#pragma unroll
            for (int e = 0; e < 8; ++e) bv[e] = W2b[(ks * 32 + 8 * grp + e) * LH + t * 16 + col];
            dh[t] = mfma32(av, bv, dh[t]);
        }
    }
    // dA1 = dH1 [H1 > 0] (H1 > 0 read from its bf16 copy), into D2 / D2b
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int mm = 4 * grp + e, nn = t * 16 + col;
            const float hv = __uint_as_float(((uint32_t)(uint16_t)Hw[mm * LH + nn]) << 16);
            const float v = hv > 0.f ? dh[t][e] : 0.f;
            D2[mm * LH + nn] = v;
            D2b[mm * LH + nn] = f2bf(v);
        }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int nn = lane; nn < LH; nn += 64) {
        float s = 0.f;
        for (int mm = 0; mm < 16; ++mm) s += D2[mm * LH + nn];
        atomicAdd(&grad[MLP_B1 + nn], s);
    }
    // dW1[o][i] = sum_m dA1[m][o] X[m][i]: A = dA1^T (M = o, K = m), B = X (K = m, N = i)
    for (int to = 0; to < 8; ++to) {
        bf16x4 av;
#pragma unroll
        for (int e = 0; e < 4; ++e) av[e] = D2b[(4 * grp + e) * LH + to * 16 + col];
#pragma unroll
        for (int ti = 0; ti < LIN / 16; ++ti) {
            bf16x4 bv;
#pragma unroll
            for (int e = 0; e < 4; ++e) bv[e] = Xw[(4 * grp + e) * LIN + ti * 16 + col];
            f32x4 c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
            for (int e = 0; e < 4; ++e) atomicAdd(&grad[(to * 16 + 4 * grp + e) * LIN + ti * 16 + col], c[e]);
        }
    }
}

// Adam on the FP32 master parameters; refreshes the BF16 weight copies and
// the FP64 copy, and clears the gradient for the next step
__global__ __launch_bounds__(256) void k_adam(LearnArgs g, float* grad, float* m, float* v, float lr, float c1,
                                              float c2)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= MLP_PARAMS) return;
    const float gr = grad[i];
    const float mi = 0.9f * m[i] + 0.1f * gr;
    const float vi = 0.999f * v[i] + 0.001f * gr * gr;
    m[i] = mi;
    v[i] = vi;
    const float p = g.p32[i] - lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
    g.p32[i] = p;
    g.p64[i] = (double)p;
    if (i < MLP_B1) g.w1b[i] = f2bf(p);
    else if (i >= MLP_W2 && i < MLP_B2) g.w2b[i - MLP_W2] = f2bf(p);
    grad[i] = 0.f;
}

// parameters (FP32) -> BF16 weight copies and FP64 copy
__global__ __launch_bounds__(256) void k_params_convert(LearnArgs g)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= MLP_PARAMS) return;
    const float p = g.p32[i];
    g.p64[i] = (double)p;
    if (i < MLP_B1) g.w1b[i] = f2bf(p);
    else if (i >= MLP_W2 && i < MLP_B2) g.w2b[i - MLP_W2] = f2bf(p);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
size_t learn_lds_bytes() { return sizeof(short) * (LH * LIN + LH * LH + 4 * 16 * LIN + 4 * 16 * LH); }

size_t grad_lds_bytes()
{
    return learn_lds_bytes() + sizeof(float) * (8 * 16 * LH) + sizeof(short) * (4 * 16 * LH);
}

hipError_t set_learn_lds_limit()
{
    hipError_t e = hipFuncSetAttribute((const void*)k_learn<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)learn_infer_lds_bytes());
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_learn<double>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)learn_stage_bytes());
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_mlp_fwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)learn_lds_bytes());
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_mlp_grad, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)grad_lds_bytes());
    return e;
}

hipError_t launch_learn(const SweepArgs& a, const LearnArgs& g, hipStream_t s)
{
    if (a.precision == 64 || !g.infer)
        hipLaunchKernelGGL(k_learn<double>, dim3(g.grid), dim3(LEARN_THREADS), learn_stage_bytes(), s, a, g);
    else
        hipLaunchKernelGGL(k_learn<float>, dim3(g.grid), dim3(LEARN_THREADS), learn_infer_lds_bytes(), s, a, g);
    return hipGetLastError();
}

hipError_t launch_mlp_fwd(const LearnArgs& g, const float* X, int nrows, float* out, hipStream_t s)
{
    if (nrows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_fwd, dim3((nrows + 63) / 64), dim3(256), learn_lds_bytes(), s, g, X, nrows, out);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const LearnArgs& g, const float* data, const int* rows, int nrows, float inv_batch,
                           float* grad, double* loss, hipStream_t s)
{
    if (nrows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_grad, dim3((nrows + 63) / 64), dim3(256), grad_lds_bytes(), s, g, data, rows, nrows,
                       inv_batch, grad, loss);
    return hipGetLastError();
}

hipError_t launch_adam(const LearnArgs& g, float* grad, float* m, float* v, float lr, float c1, float c2,
                       hipStream_t s)
{
    hipLaunchKernelGGL(k_adam, dim3((MLP_PARAMS + 255) / 256), dim3(256), 0, s, g, grad, m, v, lr, c1, c2);
    return hipGetLastError();
}

hipError_t launch_params_convert(const LearnArgs& g, hipStream_t s)
{
    hipLaunchKernelGGL(k_params_convert, dim3((MLP_PARAMS + 255) / 256), dim3(256), 0, s, g);
    return hipGetLastError();
}

} // namespace crmc

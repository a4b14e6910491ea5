// CDNA4 (gfx950) kernels of the learned site proposal.
//
//   k_learn      per colour phase: for the sites of every active cell, the
//                environment features (charged particles of the 26 neighbour
//                cells within rc, by radial shell and sign relative to the
//                site's ionized charge), appended to the phase's list; and
//                optionally one labelled training row per site.
//   k_mlp_infer<R> per colour phase: the network output p = logistic of a
//                32 -> 128 -> 128 -> 1 ReLU perceptron for every listed site.
//                R = float: BF16 matrix cores (v_mfma_f32_16x16x16bf16_1k)
//                with FP32 accumulation; R = double: FP64, vector unit.
//   k_mlp_grad   mean binary cross-entropy gradient of a minibatch on the
//                matrix cores (BF16 operands, FP32 accumulation).
//   k_adam       Adam step on the FP32 master parameters, refreshing the
//                BF16 copies the inference uses.
//   k_mlp_fwd    logits of given feature rows (same path as k_learn).
//
// The neighbour cells are inactive during the phase, so the outputs fix the
// proposal weights of the phase's trials (detailed balance holds for the
// frozen environment).
#include "crmc_internal.h"

namespace crmc {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int LIN = MLP_IN, LH = MLP_H;
constexpr int SITES_PER_WG = 64;    // sites of one cell handled by one workgroup
constexpr int STAGE = 1024;         // neighbour records staged per round

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
// Returns the logit of row (lane & 15) in every lane of that row group.
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
    for (int ks = 0; ks < LIN / 16; ++ks) {
        bf16x4 a;
#pragma unroll
        for (int e = 0; e < 4; ++e) a[e] = X[col * LIN + ks * 16 + 4 * grp + e];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            bf16x4 b;
#pragma unroll
            for (int e = 0; e < 4; ++e) b[e] = W1b[(t * 16 + col) * LIN + ks * 16 + 4 * grp + e];
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
        }
    }
    // bias, ReLU, to LDS as bf16 (row-major [m][n])
#pragma unroll
    for (int t = 0; t < 8; ++t)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int m = 4 * grp + e, n = t * 16 + col;
            const float v = acc[t][e] + b1[n];
            H[m * LH + n] = f2bf(v > 0.f ? v : 0.f);
        }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // layer 2: D[m][n] = sum_k H1[m][k] W2[n][k]
#pragma unroll
    for (int t = 0; t < 8; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int ks = 0; ks < LH / 16; ++ks) {
        bf16x4 a;
#pragma unroll
        for (int e = 0; e < 4; ++e) a[e] = H[col * LH + ks * 16 + 4 * grp + e];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            bf16x4 b;
#pragma unroll
            for (int e = 0; e < 4; ++e) b[e] = W2b[(t * 16 + col) * LH + ks * 16 + 4 * grp + e];
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[t], 0, 0, 0);
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
// k_learn: features and site probabilities of the active sites of a phase
// ---------------------------------------------------------------------------
struct LearnShared {
    uint4 site[SITES_PER_WG];    // x, y, z, meta of this workgroup's sites
    int hist[SITES_PER_WG][LIN]; // feature counts
    uint4 nb[STAGE];             // staged charged neighbours: x, y, z, charge
    int seg[27];                 // prefix of the 26 neighbour counts
    uint32_t segcell[26];
    int nsite, nstaged;
    uint32_t slot0;
    uint64_t r2sh[17];
};

__global__ __launch_bounds__(256) void k_learn(SweepArgs a, LearnArgs g)
{
    __shared__ LearnShared S;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t act = blockIdx.x, part = blockIdx.y;
    const uint32_t r = g.act2rep[act];
    const Replica& R = a.reps[r];
    const uint32_t n = R.n, h = R.h, cap = R.cap;
    const int colour = a.colour;
    const uint32_t px = colour & 1, py = (colour >> 1) & 1, pz = (colour >> 2) & 1;
    const uint32_t m = act - R.act_begin;
    const uint32_t cx = 2u * (m % h) + px, cy = 2u * ((m / h) % h) + py, cz = 2u * (m / (h * h)) + pz;
    const uint32_t cell = cx + n * (cy + n * cz);
    const uint64_t s = *a.sweep;
    const int buf = (int)((s + 1u) & 1u);
    const uint4* recb = R.rec[buf];
    const uint32_t* cntb = R.cnt[buf];
    const int nown = (int)cntb[cell];
    // a cell with at most part*64 records has no sites for this workgroup
    if (nown <= (int)part * SITES_PER_WG) return;

    // this workgroup's share of the cell's sites: sites part*64 .. part*64+63
    if (tid == 0) S.nsite = 0;
    __syncthreads();
    {
        int base = 0;
        for (int b0 = 0; b0 < nown; b0 += 256) {
            const int i = b0 + tid;
            uint4 v = make_uint4(0, 0, 0, 0);
            bool site = false;
            if (i < nown) {
                v = recb[(size_t)cell * cap + i];
                const uint32_t k = v.w & 7u;
                site = k == KIND_ACID || k == KIND_BASE;
            }
            // rank among the sites (block-wide prefix through the wave ballots)
            __shared__ int wcount[4];
            const uint64_t mask = __ballot(site);
            if (lane == 0) wcount[wave] = __popcll(mask);
            __syncthreads();
            int before = base;
            for (int w = 0; w < wave; ++w) before += wcount[w];
            const int rank = before + __popcll(mask & lanes_below());
            const int lo = (int)part * SITES_PER_WG;
            if (site && rank >= lo && rank < lo + SITES_PER_WG) S.site[rank - lo] = v;
            int tot = 0;
            for (int w = 0; w < 4; ++w) tot += wcount[w];
            base += tot;
            __syncthreads();
        }
        if (tid == 0) {
            const int lo = (int)part * SITES_PER_WG;
            S.nsite = base <= lo ? 0 : min(SITES_PER_WG, base - lo);
        }
    }
    __syncthreads();
    const int nsite = S.nsite;
    if (nsite == 0) return;
    for (int i = tid; i < SITES_PER_WG * LIN; i += 256) (&S.hist[0][0])[i] = 0;
    // neighbour segments
    if (tid < 26) {
        const int oo = tid < 13 ? tid : tid + 1;
        const uint32_t x = (cx + n + (uint32_t)(oo % 3) - 1u) % n, y = (cy + n + (uint32_t)((oo / 3) % 3) - 1u) % n,
                       z = (cz + n + (uint32_t)(oo / 9) - 1u) % n;
        S.segcell[tid] = x + n * (y + n * z);
    }
    __syncthreads();
    if (tid == 0) {
        int acc = 0;
        for (int q = 0; q < 26; ++q) { S.seg[q] = acc; acc += (int)cntb[S.segcell[q]]; }
        S.seg[26] = acc;
    }
    if (tid < 17) S.r2sh[tid] = g.R2sh[(size_t)r * 17 + tid];
    __syncthreads();
    const int nbt = S.seg[26];
    const uint64_t* R2sh = S.r2sh;
    const uint64_t R2 = R2sh[16];
    // shell k holds sqrt(d2) / c in [k, k + 1) with c = rc / 16 in lattice
    // units; the float quotient decides unless it lies within 1e-4 of an
    // integer, where the exact integer thresholds do
    const float inv_c = 16.0f / sqrtf((float)R2);

    // rounds of staged charged neighbours; lane = site, waves split the records
    for (int r0 = 0; r0 < nbt; r0 += STAGE) {
        if (tid == 0) S.nstaged = 0;
        __syncthreads();
        for (int i = r0 + tid; i < min(nbt, r0 + STAGE); i += 256) {
            int q = 0, hi = 26; // seg[q] <= i < seg[hi]
            while (hi - q > 1) {
                const int mid = (q + hi) >> 1;
                if (S.seg[mid] <= i) q = mid; else hi = mid;
            }
            const uint4 v = recb[(size_t)S.segcell[q] * cap + (uint32_t)(i - S.seg[q])];
            const int qq = q_of(v.w);
            if (qq != 0) {
                const int slot = atomicAdd(&S.nstaged, 1);
                S.nb[slot] = make_uint4(v.x, v.y, v.z, (uint32_t)qq);
            }
        }
        __syncthreads();
        const int ns = S.nstaged;
        if (lane < nsite) {
            const uint4 me = S.site[lane];
            const int qion = (me.w & 7u) == KIND_ACID ? -1 : 1;
            for (int j = wave; j < ns; j += 4) {
                const uint4 o = S.nb[j];
                const int32_t dx = (int32_t)(o.x - me.x), dy = (int32_t)(o.y - me.y), dz = (int32_t)(o.z - me.z);
                const float fx = (float)dx, fy = (float)dy, fz = (float)dz;
                const float t = sqrtf(fx * fx + fy * fy + fz * fz) * inv_c;
                if (!(t < 16.0001f)) continue;
                int k = (int)t;
                const float fr = t - (float)k;
                if (fr < 1e-4f || fr > 0.9999f) {
                    // near a shell boundary or the cutoff: exact integer thresholds
                    const uint32_t ax = (uint32_t)abs(dx), ay = (uint32_t)abs(dy), az = (uint32_t)abs(dz);
                    const uint64_t d2 = (uint64_t)ax * ax + (uint64_t)ay * ay + (uint64_t)az * az;
                    if (d2 >= R2) continue;
                    k = k > 15 ? 15 : k;
                    while (k > 0 && d2 < R2sh[k]) --k;
                    while (k < 15 && d2 >= R2sh[k + 1]) ++k;
                }
                const int ch = ((int)o.w * qion < 0) ? 0 : 16;
                atomicAdd(&S.hist[lane][ch + k], 1);
            }
        }
        __syncthreads();
    }

    // training rows: features and the site's ionization at the start of the phase
    if (g.data && tid < nsite) {
        const unsigned long long row = atomicAdd(g.data_n, 1ull);
        if (row < g.data_cap) {
            for (int i = 0; i < LIN; ++i) g.data[row * (LIN + 1) + i] = (float)S.hist[tid][i];
            g.data[row * (LIN + 1) + LIN] = (float)((S.site[tid].w >> 3) & 1u);
        }
    }
    if (!g.infer) return;
    // the phase's list of sites for the network: (replica, site id), features
    if (tid == 0) S.slot0 = atomicAdd(&g.list_n[colour], (uint32_t)nsite);
    __syncthreads();
    for (int i = tid; i < nsite * LIN; i += 256) {
        const uint32_t slot = S.slot0 + (uint32_t)(i / LIN);
        if (slot < g.list_cap) g.feat[(size_t)slot * LIN + i % LIN] = (float)S.hist[i / LIN][i % LIN];
    }
    if (tid < nsite && S.slot0 + (uint32_t)tid < g.list_cap) g.list[S.slot0 + tid] = make_uint2(r, S.site[tid].w >> 8);
}

// network outputs of the listed sites of a phase: 64 per workgroup
template <typename Real>
__global__ __launch_bounds__(256) void k_mlp_infer(SweepArgs a, LearnArgs g)
{
    extern __shared__ short lsh[]; // bf16 weights, then per-wave X and H tiles (FP32 path)
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t nlist = min(g.list_n[a.colour], g.list_cap);
    const uint32_t b0 = blockIdx.x * 64u;
    if (b0 >= nlist) return;
    const int nrow = (int)min(64u, nlist - b0);
    if (sizeof(Real) == 8) {
        if (tid < nrow) {
            double x[LIN];
            for (int i = 0; i < LIN; ++i) x[i] = (double)g.feat[(size_t)(b0 + tid) * LIN + i];
            const uint2 e = g.list[b0 + tid];
            a.reps[e.x].phat[e.y] = site_prob(mlp_row_f64(g.p64, x));
        }
        return;
    }
    short* W1b = lsh;
    short* W2b = W1b + LH * LIN;
    short* Xw = W2b + LH * LH + wave * (16 * LIN);
    short* Hw = W2b + LH * LH + 4 * 16 * LIN + wave * (16 * LH);
    for (int i = tid; i < LH * LIN; i += 256) W1b[i] = g.w1b[i];
    for (int i = tid; i < LH * LH; i += 256) W2b[i] = g.w2b[i];
    __syncthreads();
    const int row0 = wave * 16;
    if (row0 >= nrow) return;
    for (int i = lane; i < 16 * LIN; i += 64) {
        const int rr = row0 + i / LIN;
        Xw[i] = rr < nrow ? f2bf(g.feat[(size_t)(b0 + rr) * LIN + i % LIN]) : (short)0;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    const float z = mlp_rows16(W1b, W2b, g.p32 + MLP_B1, g.p32 + MLP_B2, g.p32 + MLP_W3, g.p32[MLP_B3], Xw, Hw,
                               nullptr);
    const int rr = row0 + (lane & 15);
    if (lane < 16 && rr < nrow) {
        const uint2 e = g.list[b0 + rr];
        a.reps[e.x].phat[e.y] = site_prob((double)z);
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
    for (int ks = 0; ks < LH / 16; ++ks) {
        bf16x4 av;
#pragma unroll
        for (int e = 0; e < 4; ++e) av[e] = D2b[col * LH + ks * 16 + 4 * grp + e];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            bf16x4 bv;
#pragma unroll
            for (int e = 0; e < 4; ++e) bv[e] = W2b[(ks * 16 + 4 * grp + e) * LH + t * 16 + col];
            dh[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, dh[t], 0, 0, 0);
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
    hipError_t e = hipFuncSetAttribute((const void*)k_mlp_infer<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)learn_lds_bytes());
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
    hipLaunchKernelGGL(k_learn, dim3(g.nact_total, g.parts), dim3(256), 0, s, a, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !g.infer) return e;
    const dim3 grid((g.list_cap + 63u) / 64u);
    if (a.precision == 64)
        hipLaunchKernelGGL(k_mlp_infer<double>, grid, dim3(256), 0, s, a, g);
    else
        hipLaunchKernelGGL(k_mlp_infer<float>, grid, dim3(256), learn_lds_bytes(), s, a, g);
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

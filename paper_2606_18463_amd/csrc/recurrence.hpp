// The s-step residual-correction recurrence (Algorithm 1, inner loop, with
// the L2 decay) spread over several workgroups of one launch.
//
//   z_j = beta^j r_j + alpha sum_{i<j} beta^(j-1-i) G_{j,i} delta_i,
//   delta_j = glm_delta(z_j, y_j) (logistic: y_j / (1 + exp(y_j z_j))),
//   c_j = beta^(s-1-j) delta_j.
//
// The chain over j is sequential, but G is known before it starts. The main
// workgroup (blockIdx 0) runs the chain and adds only the last W column
// blocks itself ("near" part: G_{j,i} for j-W <= i < j, loaded while it waits
// for the rest). Helper workgroup k (k = 1 .. s-W-1) owns row block
// j = W + k and accumulates its "far" part sum_{i<j-W} as the deltas arrive;
// it has W steps of the chain to deliver it. The two sides exchange values
// through tagged 64-bit words in the workspace (value bits in the low half,
// the tag in the high half, written and read with single-copy-atomic
// relaxed accesses), so no fence or cache write-back is needed: a reader
// simply waits until the word carries the current tag. The main workgroup
// clears the words once the chain is done, so every launch starts from zero.
#pragma once

#include "dense.hpp"

namespace casgd {

constexpr unsigned kPubTag = 1u;

template <typename ACC>
constexpr int pub_words() { return sizeof(ACC) / 4; }

__device__ __forceinline__ void pub_put(unsigned long long* p, float v) {
    __hip_atomic_store(p, ((unsigned long long)kPubTag << 32) | __float_as_uint(v),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void pub_put(unsigned long long* p, double v) {
    const unsigned long long bits = (unsigned long long)__double_as_longlong(v);
    __hip_atomic_store(p, ((unsigned long long)kPubTag << 32) | (bits & 0xffffffffull),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(p + 1, ((unsigned long long)kPubTag << 32) | (bits >> 32),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long pub_word(const unsigned long long* p) {
    return __hip_atomic_load(const_cast<unsigned long long*>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool pub_get(const unsigned long long* p, float& v) {
    const unsigned long long x = pub_word(p);
    if ((unsigned)(x >> 32) != kPubTag) return false;
    v = __uint_as_float((unsigned)x);
    return true;
}
__device__ __forceinline__ bool pub_get(const unsigned long long* p, double& v) {
    const unsigned long long lo = pub_word(p), hi = pub_word(p + 1);
    if ((unsigned)(lo >> 32) != kPubTag || (unsigned)(hi >> 32) != kPubTag) return false;
    v = __longlong_as_double((long long)((hi << 32) | (lo & 0xffffffffull)));
    return true;
}

// Bounded wait for a tagged value. Returns false (after raising the timeout
// flag) when the spin limit is reached or another workgroup timed out.
template <typename ACC>
__device__ __forceinline__ bool pub_wait(const unsigned long long* p, ACC& v, unsigned* flags,
                                         unsigned long long spin) {
    unsigned long long n = 0;
    while (!pub_get(p, v)) {
        if (++n > spin) {
            raise_flag(flags, FLAG_TIMEOUT);
            return false;
        }
        if ((n & 63ull) == 0 && atomic_load_relaxed(flags + FLAG_TIMEOUT)) return false;
        __builtin_amdgcn_s_sleep(1);
    }
    return true;
}

// Near-block window W for b = 16 * NV. The exchange with a helper takes
// about one chain step, so two near blocks hide it; every extra block costs
// the chain LDS reads and FMAs on its critical path (measured on MI355X:
// W = 2 is fastest for b = 64 at s = 4 .. 32). b = 128 needs two row passes
// and keeps one block (registers: two sets of PASSES * W * NV float4).
template <int NV>
constexpr int rec_passes() { return NV <= 4 ? 1 : NV / 4; }
template <int NV>
constexpr int rec_window() { return NV <= 4 ? 2 : 1; }

// dot of NV float4 of G with 4*NV consecutive deltas in LDS
template <typename ACC, int NV>
__device__ __forceinline__ ACC dot_nv(const float4 (&g)[NV], const ACC* d) {
    ACC a = 0;
#pragma unroll
    for (int v = 0; v < NV; ++v)
        a += (ACC)g[v].x * d[4 * v] + (ACC)g[v].y * d[4 * v + 1] + (ACC)g[v].z * d[4 * v + 2] +
             (ACC)g[v].w * d[4 * v + 3];
    return a;
}

// Helper workgroups of the recurrence for block size b (b = 16, 32, 64, 128).
__host__ __device__ inline int rec_helpers(int b, int s) {
    const int w = b <= 64 ? 2 : 1;   // rec_window<b / 16>()
    return s - w - 1 > 0 ? s - w - 1 : 0;
}

// The recurrence for b = 16 * NV on 1 + rec_helpers(b, s) workgroups of kNT
// threads, all resident; `rank` is this workgroup's index among them. Thread layout: four
// threads per row (sub = tid % 4 owns columns [sub*b/4, (sub+1)*b/4) of
// every column block), 64 rows per pass. r: reduced margins (row scales
// applied); y: labels; c, delta_out: outputs; pub: 2 * sb * pub_words
// tagged words (deltas, then far sums).
template <typename ACC, int NV, int W = rec_window<NV>(), bool GEN = true>
__device__ void recurrence_multi(const Dense& P, const float* G, const float* r, const float* y,
                                 float* c, float* delta_out, unsigned long long* pub,
                                 unsigned long long spin, unsigned char* lds, int rank) {
    constexpr int PASSES = rec_passes<NV>();
    constexpr int PW = pub_words<ACC>();
    const int b = 16 * NV, s = P.s, sb = P.sb;
    const int tid = threadIdx.x, sub = tid & 3, rho = tid >> 2;
    const int cb = sub * 4 * NV;   // first column of this thread within a block
    ACC* dl = reinterpret_cast<ACC*>(lds);        // sb deltas (main) / b deltas (helper)
    ACC* pw = dl + sb;                            // beta^0 .. beta^s
    __shared__ int s_stop;
    unsigned long long* dpub = pub;
    unsigned long long* fpub = pub + (size_t)sb * PW;
    const ACC alpha = (ACC)P.alpha_d;
    if (tid == 0) {
        ACC p = 1;
        const ACC be = (ACC)P.beta_d;
        for (int k = 0; k <= s; ++k) { pw[k] = p; p *= be; }
        s_stop = 0;
    }
    __syncthreads();
    const int R = s - W - 1 > 0 ? s - W - 1 : 0;

    if (rank == 0) {
        // ------------------------------------------------------------ main
        // Step j uses the near blocks and far-sum words loaded during step
        // j-1 (two register sets, alternating), so their latency overlaps a
        // whole step.
        float4 gA[PASSES][W][NV], gB[PASSES][W][NV];
        unsigned long long fA[PASSES][PW], fB[PASSES][PW];
        float2 ryA[PASSES], ryB[PASSES];   // margin and label of the row
        // Loads are unconditional (indices clamped into range, unused values
        // ignored): a conditional load becomes a branch, and the join would
        // wait for it.
        auto load_next = [&](float4 (&g)[PASSES][W][NV], unsigned long long (&f)[PASSES][PW],
                             float2 (&ry)[PASSES], int j) {
            const int jj = j < s ? j : s - 1;
#pragma unroll
            for (int p = 0; p < PASSES; ++p) {
                const int q = p * 64 + rho;
                const int t = jj * b + (q < b ? q : b - 1);
                const float* grow = G + (int64_t)t * P.ldg + cb;
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    const int i = j - W + k;
                    const int ii = i > 0 ? i : 0;
#pragma unroll
                    for (int v = 0; v < NV; ++v)
                        g[p][k][v] = *reinterpret_cast<const float4*>(grow + (int64_t)ii * b + 4 * v);
                }
#pragma unroll
                for (int w = 0; w < PW; ++w) f[p][w] = pub_word(fpub + (size_t)t * PW + w);
                ry[p] = make_float2(r[t], y[t]);
            }
        };
        auto step = [&](const float4 (&g)[PASSES][W][NV], const unsigned long long (&f)[PASSES][PW],
                        const float2 (&ry)[PASSES], int j) {
#pragma unroll
            for (int p = 0; p < PASSES; ++p) {
                const int q = p * 64 + rho;
                // far part from the helper of this block (already loaded, or wait)
                ACC far = 0;
                if (j > W && sub == 0 && q < b) {
                    bool ok = (unsigned)(f[p][0] >> 32) == kPubTag &&
                              (unsigned)(f[p][PW - 1] >> 32) == kPubTag;
                    if (ok) {
                        if constexpr (PW == 1) {
                            far = (ACC)__uint_as_float((unsigned)f[p][0]);
                        } else {
                            far = (ACC)__longlong_as_double(
                                (long long)((f[p][PW - 1] << 32) | (f[p][0] & 0xffffffffull)));
                        }
                    } else if (!pub_wait(fpub + (size_t)(j * b + q) * PW, far, P.flags, spin)) {
                        s_stop = 1;
                    }
                }
                ACC nsum = 0;
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    const int i = j - W + k;
                    if (i >= 0) nsum += pw[j - 1 - i] * dot_nv<ACC, NV>(g[p][k], dl + i * b + cb);
                }
                nsum += shfl_xor(nsum, 1);
                nsum += shfl_xor(nsum, 2);
                if (sub == 0 && q < b) {
                    const int t = j * b + q;
                    const ACC rv = (ACC)ry[p].x, yv = (ACC)ry[p].y;
                    const int e2e = e2e_mode<GEN>(P);
                    const ACC z = e2e_round(pw[j] * rv + alpha * e2e_round(far + nsum, e2e), e2e);
                    const ACC d = e2e_round(glm_delta<ACC>(z, yv, loss_mode<GEN>(P)), e2e);
                    if (!isfinite(z) || !isfinite(d)) raise_flag(P.flags, FLAG_NONFINITE);
                    dl[t] = d;
                    c[t] = (float)e2e_round(pw[s - 1 - j] * d, e2e);
                    if (delta_out) delta_out[t] = (float)d;
                    if (j < R) pub_put(dpub + (size_t)t * PW, d);
                }
            }
            lds_barrier();
        };
        load_next(gA, fA, ryA, 0);
        for (int j = 0; j < s; j += 2) {
            load_next(gB, fB, ryB, j + 1);
            step(gA, fA, ryA, j);
            if (s_stop) return;
            if (j + 1 < s) {
                load_next(gA, fA, ryA, j + 2);
                step(gB, fB, ryB, j + 1);
                if (s_stop) return;
            }
        }
        // every helper has delivered its far sums, hence read all deltas it
        // needs: clear the words for the next launch
        for (int k = tid; k < 2 * sb * PW; k += blockDim.x) pub[k] = 0ull;
        return;
    }

    // ------------------------------------------------------------ helpers
    const int jh = W + rank;                 // the row block this helper owns
    if (jh >= s) return;
    ACC* di = dl;                            // deltas of the current column block
    ACC acc[PASSES];
#pragma unroll
    for (int p = 0; p < PASSES; ++p) acc[p] = 0;
    for (int i = 0; i < jh - W; ++i) {
        float4 g[PASSES][NV];
#pragma unroll
        for (int p = 0; p < PASSES; ++p) {
            const int q = p * 64 + rho;
            const float* grow = G + (int64_t)(jh * b + (q < b ? q : b - 1)) * P.ldg + (int64_t)i * b + cb;
#pragma unroll
            for (int v = 0; v < NV; ++v) g[p][v] = *reinterpret_cast<const float4*>(grow + 4 * v);
        }
        if (tid < b) {
            ACC d;
            if (pub_wait(dpub + (size_t)(i * b + tid) * PW, d, P.flags, spin)) di[tid] = d;
            else s_stop = 1;
        }
        lds_barrier();
        if (s_stop) return;
#pragma unroll
        for (int p = 0; p < PASSES; ++p) acc[p] += pw[jh - 1 - i] * dot_nv<ACC, NV>(g[p], di + cb);
        lds_barrier();
    }
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
        const int q = p * 64 + rho;
        ACC a = acc[p];
        a += shfl_xor(a, 1);
        a += shfl_xor(a, 2);
        if (sub == 0 && q < b) pub_put(fpub + (size_t)(jh * b + q) * PW, a);
    }
}

}  // namespace casgd

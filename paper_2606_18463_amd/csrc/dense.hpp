// Device functions of the dense s-step SGD outer iteration (Algorithm 1 with
// L2 decay) for gfx950. Used both by the one-launch-per-phase kernels and by
// the persistent fused kernel.
#pragma once

#include "common.hpp"

namespace casgd {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr int kTile = 64;   // Gram tile edge in sampled rows
constexpr int kLPR = 8;     // lanes per row in the update / margin passes

// One dense problem: inputs, scalars, launch geometry and workspace views.
struct Dense {
    const void* X;
    const float* scale;     // row scales or nullptr
    const float* y;
    float* x;
    int64_t m, n, ld;
    int b, s, sb;
    uint64_t seed;
    float alpha, beta, beta_s;        // alpha = eta/b, beta = 1 - eta*lambda
    double alpha_d, beta_d;
    int ts;                 // tiles per side = ceil(sb / kTile)
    int ntiles;             // ts (ts + 1) / 2 lower-triangular tiles
    int ksplit;             // K splits per tile
    int64_t kchunk;         // K elements per split (multiple of the K step)
    int nslices;            // column slices of the update / margin passes
    unsigned* flags;        // FLAG_* words
    unsigned* tile_cnt;     // split-K arrival counters, one per tile
    float* G[2];            // sb x sb, row-major, strict block-lower part used
    float* Gpart;           // ntiles * ksplit * 4096 split-K partial tiles
    float* rp[2];           // nslices x sb partial margins
    float* c;               // sb corrected residual weights
    float* x_hist;          // snapshots or nullptr
    int64_t* t_hist;        // snapshot clocks or nullptr
    int64_t snap_every;
};

// Sum over groups of G consecutive lanes, G a power of two chosen at run time.
template <typename T>
__device__ __forceinline__ T group_sum_rt(T v, int G) {
    for (int off = 1; off < G; off <<= 1) v += shfl_xor(v, off);
    return v;
}

// Threads per row of the recurrence: the largest power of two with
// tpr * b <= NT, at least 1 and at most 64 (one wave).
__host__ __device__ inline int recurrence_tpr(int NT, int b) {
    int t = 1;
    while (t < 64 && 2 * t * b <= NT) t *= 2;
    return t;
}

// Column-slice width of the update / margin passes for a storage type.
template <int DT>
constexpr int slice_width() { return kLPR * Store<DT>::kVec; }

// ------------------------------------------------------------------ Gram
// Tile p of the lower triangle (TJ >= TI) in row-major triangular order.
__device__ __forceinline__ void tile_coords(int p, int& TJ, int& TI) {
    int j = (int)((sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
    while (j * (j + 1) / 2 > p) --j;
    while ((j + 1) * (j + 2) / 2 <= p) ++j;
    TJ = j;
    TI = p - j * (j + 1) / 2;
}

// A tile holds strict block-lower entries iff its first column lies in an
// earlier block than its last row.
__device__ __forceinline__ bool tile_needed(const Dense& P, int TJ, int TI) {
    const int rlast = min(TJ * kTile + kTile - 1, P.sb - 1);
    return (TI * kTile) / P.b < rlast / P.b;
}

template <int DT>
__device__ __forceinline__ void mfma_step(const V16& a, const V16& b, v4f& acc) {
    if constexpr (DT == DT_F32) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w[q]),
                                                       __uint_as_float(b.w[q]), acc, 0, 0, 0);
    } else if constexpr (DT == DT_BF16) {
        bf16x8 av, bv;
        __builtin_memcpy(&av, &a, 16);
        __builtin_memcpy(&bv, &b, 16);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
    } else if constexpr (DT == DT_F16) {
        f16x8 av, bv;
        __builtin_memcpy(&av, &a, 16);
        __builtin_memcpy(&bv, &b, 16);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, acc, 0, 0, 0);
    } else {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const long av = (long)(((uint64_t)a.w[2 * q + 1] << 32) | a.w[2 * q]);
            const long bv = (long)(((uint64_t)b.w[2 * q + 1] << 32) | b.w[2 * q]);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, bv, acc, 0, 0, 0);
        }
    }
}

// Write one 64x64 tile held as 4x4 MFMA 16x16 sub-tiles. With the 16x16
// MFMA output layout, lane l and register v hold row 4*(l/16)+v, column l%16
// of a sub-tile. Only strict block-lower entries inside sb x sb are stored;
// row scales (if any) are applied here.
__device__ __forceinline__ void store_tile(const Dense& P, float* Gout, int TJ, int TI,
                                           const v4f (&acc)[4][4], const float (&sr)[4][4],
                                           const float (&sc)[4]) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lg = lane >> 4;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int t = TJ * kTile + 16 * a + 4 * lg + v;
            if (t >= P.sb) continue;
            const int bt = t / P.b;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int u = TI * kTile + 16 * c + li;
                if (u < P.sb && u / P.b < bt)
                    Gout[(int64_t)t * P.sb + u] = acc[a][c][v] * sr[a][v] * sc[c];
            }
        }
    }
}

// One work item = one K split of one 64x64 tile, computed by one wave with
// operands loaded straight from the sampled rows of X into registers (both
// MFMA operands are K-contiguous rows of Y, so no LDS transpose is needed).
// Lane l owns row l%16 of each 16-row sub-tile and the 16-byte K segment
// (l/16); within a K step every (lane group, vector element) pair maps to a
// distinct k, identically for both operands, so the products pair up.
template <int DT>
__device__ void gram_item(const Dense& P, float* Gout, uint64_t h, int item) {
    using T = typename Store<DT>::T;
    constexpr int VEC = Store<DT>::kVec;
    constexpr int KSTEP = 4 * VEC;
    const int lane = threadIdx.x & 63;
    const int tile = item / P.ksplit;
    const int split = item - tile * P.ksplit;
    int TJ, TI;
    tile_coords(tile, TJ, TI);
    if (!tile_needed(P, TJ, TI)) return;
    const bool diag = TJ == TI;
    const int li = lane & 15, lg = lane >> 4;
    const T* X = static_cast<const T*>(P.X);
    const uint64_t t0 = h * (uint64_t)P.sb;

    const T* ra[4];
    const T* rb[4];
    bool va[4], vb[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int t = TJ * kTile + 16 * a + li;
        va[a] = t < P.sb;
        ra[a] = X + (va[a] ? sample_row(P.seed, t0 + t, P.m) : 0) * P.ld;
        const int u = TI * kTile + 16 * a + li;
        vb[a] = u < P.sb;
        rb[a] = X + (vb[a] ? sample_row(P.seed, t0 + u, P.m) : 0) * P.ld;
    }

    const int64_t k0 = (int64_t)split * P.kchunk;
    const int64_t k1 = min(P.n, k0 + P.kchunk);
    v4f acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = v4f{0.f, 0.f, 0.f, 0.f};

    const V16 zero = {{0u, 0u, 0u, 0u}};
    V16 A[4], B[4], An[4], Bn[4];
    auto load = [&](V16 (&Av)[4], V16 (&Bv)[4], int64_t k) {
        const int64_t kk = k + VEC * lg;
#pragma unroll
        for (int a = 0; a < 4; ++a) Av[a] = va[a] ? load_v16<DT>(ra[a], kk, P.n) : zero;
        if (!diag) {
#pragma unroll
            for (int c = 0; c < 4; ++c) Bv[c] = vb[c] ? load_v16<DT>(rb[c], kk, P.n) : zero;
        }
    };
    if (k0 < k1) load(A, B, k0);
    for (int64_t k = k0; k < k1; k += KSTEP) {
        const bool more = k + KSTEP < k1;
        if (more) load(An, Bn, k + KSTEP);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < 4; ++c) mfma_step<DT>(A[a], diag ? A[c] : B[c], acc[a][c]);
        if (more) {
#pragma unroll
            for (int a = 0; a < 4; ++a) { A[a] = An[a]; B[a] = Bn[a]; }
        }
    }

    // Row scales of the tile's rows (output layout) and columns.
    float sr[4][4], sc[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int t = TJ * kTile + 16 * a + 4 * lg + v;
            sr[a][v] = (P.scale && t < P.sb) ? P.scale[sample_row(P.seed, t0 + t, P.m)] : 1.0f;
        }
        const int u = TI * kTile + 16 * a + li;
        sc[a] = (P.scale && u < P.sb) ? P.scale[sample_row(P.seed, t0 + u, P.m)] : 1.0f;
    }

    if (P.ksplit == 1) {
        store_tile(P, Gout, TJ, TI, acc, sr, sc);
        return;
    }
    // Split-K: publish this split, and let the last arriving split reduce all
    // partials in split order (deterministic) and store the tile.
    float* part = P.Gpart + ((int64_t)tile * P.ksplit + split) * 4096;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) part[((a * 4 + c) * 4 + v) * 64 + lane] = acc[a][c][v];
    __threadfence();
    unsigned prev = 0;
    if (lane == 0) prev = atomic_add_acq_rel(P.tile_cnt + tile, 1u);
    prev = __shfl(prev, 0, kWave);
    if (prev != (unsigned)P.ksplit - 1u) return;
    __threadfence();
    const float* base = P.Gpart + (int64_t)tile * P.ksplit * 4096;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = ((a * 4 + c) * 4 + v) * 64 + lane;
                float sum = 0.f;
                for (int sp = 0; sp < P.ksplit; ++sp)
                    sum += __builtin_nontemporal_load(base + (int64_t)sp * 4096 + r);
                acc[a][c][v] = sum;
            }
    store_tile(P, Gout, TJ, TI, acc, sr, sc);
    if (lane == 0) atomic_store_relaxed(P.tile_cnt + tile, 0u);
}

// ------------------------------------------------------ update and margin
// Column slice `slice` (slice_width<DT>() columns): optionally
//   x <- beta^s x + alpha * sum_t c_t * scale_t * Y_t[slice]      (outer h)
// and then optionally the partial margins of outer hn on the (new) slice:
//   rp_out[slice][t] = Y_t[slice] . x[slice]   (row scale applied later).
// A row is read by kLPR lanes with 16-byte loads; NW waves share the rows.
// Uses LDS `red` (NW * width floats) and `xs` (width floats).
template <int DT, int NW>
__device__ void update_margin_slice(const Dense& P, int slice, const float* c, uint64_t h,
                                    bool do_update, uint64_t hn, bool do_margin, float* rp_out,
                                    float* red, float* xs, int64_t snap_row) {
    using T = typename Store<DT>::T;
    constexpr int VEC = Store<DT>::kVec;
    constexpr int KW = slice_width<DT>();
    constexpr int RPW = kWave / kLPR;
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int sub = lane % kLPR, rg = lane / kLPR;
    const int64_t col0 = (int64_t)slice * KW;
    const int64_t kl = col0 + sub * VEC;
    const T* X = static_cast<const T*>(P.X);

    if (do_update) {
        const uint64_t t0 = h * (uint64_t)P.sb;
        float acc[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] = 0.f;
        for (int t = w * RPW + rg; t < P.sb; t += NW * RPW) {
            const int64_t row = sample_row(P.seed, t0 + t, P.m);
            float ct = c[t];
            if (P.scale) ct *= P.scale[row];
            const V16 v = load_v16<DT>(X + row * P.ld, kl, P.n);
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc[e] = fmaf(v16_elem<DT>(v, e), ct, acc[e]);
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            acc[e] += shfl_xor(acc[e], 8);
            acc[e] += shfl_xor(acc[e], 16);
            acc[e] += shfl_xor(acc[e], 32);
        }
        if (rg == 0) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) red[w * KW + sub * VEC + e] = acc[e];
        }
        __syncthreads();
        for (int q = tid; q < KW; q += NW * kWave) {
            const int64_t k = col0 + q;
            float xn = 0.f;
            if (k < P.n) {
                float g = 0.f;
#pragma unroll
                for (int ww = 0; ww < NW; ++ww) g += red[ww * KW + q];
                xn = P.beta_s * P.x[k] + P.alpha * g;
                P.x[k] = xn;
                if (!isfinite(xn)) raise_flag(P.flags, FLAG_NONFINITE);
                if (snap_row >= 0) P.x_hist[snap_row * P.n + k] = xn;
            }
            xs[q] = xn;
        }
        __syncthreads();
    } else {
        for (int q = tid; q < KW; q += NW * kWave) {
            const int64_t k = col0 + q;
            xs[q] = k < P.n ? P.x[k] : 0.f;
        }
        __syncthreads();
    }
    if (do_margin) {
        const uint64_t t0 = hn * (uint64_t)P.sb;
        float xv[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) xv[e] = xs[sub * VEC + e];
        for (int t = w * RPW + rg; t < P.sb; t += NW * RPW) {
            const int64_t row = sample_row(P.seed, t0 + t, P.m);
            const V16 v = load_v16<DT>(X + row * P.ld, kl, P.n);
            float d = 0.f;
#pragma unroll
            for (int e = 0; e < VEC; ++e) d = fmaf(v16_elem<DT>(v, e), xv[e], d);
            d = group_sum<kLPR>(d);
            if (sub == 0) rp_out[(int64_t)slice * P.sb + t] = d;
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------- recurrence
// The s residual corrections of one outer iteration (Algorithm 1, inner
// loop) with L2 decay, in precision ACC (the u_c slot), by one workgroup of
// NT threads. TPR threads (a power of two) cooperate on one row of a block.
//   z_t = beta^j r_t + alpha * sum_{i<j} beta^(j-1-i) (G_{t, block i} . delta_i)
//   delta_t = y_t / (1 + exp(y_t z_t));  c_t = beta^(s-1-j) delta_t
// r_t and y_t come either from the partial margins rp (summed over slices,
// times the row scale) and the sampled labels, or directly from r_in / y_in.
// Writes c (global or LDS) and optionally delta_out. Uses LDS `dl` (sb ACC)
// and `pw` (s+1 ACC).
template <typename ACC, int NT>
__device__ void recurrence(const Dense& P, const float* G, const float* rp, uint64_t h,
                           const float* r_in, const float* y_in, float* c, float* delta_out,
                           ACC* dl, ACC* pw, int TPR) {
    const int tid = threadIdx.x;
    const int b = P.b, s = P.s, sb = P.sb;
    if (tid == 0) {
        ACC p = 1;
        const ACC be = (ACC)P.beta_d;
        for (int k = 0; k <= s; ++k) { pw[k] = p; p *= be; }
    }
    __syncthreads();
    const ACC alpha = (ACC)P.alpha_d;
    const int RPP = NT / TPR;         // rows per pass
    const int sub = tid % TPR;
    const bool vec4 = (b % 4) == 0;
    const uint64_t t0 = h * (uint64_t)sb;
    for (int j = 0; j < s; ++j) {
        for (int q0 = 0; q0 < b; q0 += RPP) {
            const int q = q0 + tid / TPR;
            const bool active = q < b;
            const int t = j * b + q;
            ACC rr = 0, acc = 0;
            int64_t row = 0;
            if (active) {
                if (!r_in) {
                    row = sample_row(P.seed, t0 + t, P.m);
                    for (int sl = sub; sl < P.nslices; sl += TPR) rr += (ACC)rp[(int64_t)sl * sb + t];
                    rr = group_sum_rt(rr, TPR);
                }
                const float* grow = G + (int64_t)t * sb;
                for (int i = 0; i < j; ++i) {
                    const float* g = grow + i * b;
                    const ACC* d = dl + i * b;
                    ACC part = 0;
                    if (vec4) {
                        for (int p = 4 * sub; p < b; p += 4 * TPR) {
                            const float4 gv = *reinterpret_cast<const float4*>(g + p);
                            part += (ACC)gv.x * d[p] + (ACC)gv.y * d[p + 1] +
                                    (ACC)gv.z * d[p + 2] + (ACC)gv.w * d[p + 3];
                        }
                    } else {
                        for (int p = sub; p < b; p += TPR) part += (ACC)g[p] * d[p];
                    }
                    acc += pw[j - 1 - i] * part;
                }
                acc = group_sum_rt(acc, TPR);
            }
            if (active && sub == 0) {
                ACC r, yv;
                if (r_in) {
                    r = (ACC)r_in[t];
                    yv = (ACC)y_in[t];
                } else {
                    r = rr * (ACC)(P.scale ? P.scale[row] : 1.0f);
                    yv = (ACC)P.y[row];
                }
                const ACC z = pw[j] * r + alpha * acc;
                const ACC d = yv / ((ACC)1 + exp(yv * z));
                if (!isfinite(z)) raise_flag(P.flags, FLAG_NONFINITE);
                dl[t] = d;
                c[t] = (float)(pw[s - 1 - j] * d);
                if (delta_out) delta_out[t] = (float)d;
            }
        }
        __syncthreads();
    }
}

}  // namespace casgd

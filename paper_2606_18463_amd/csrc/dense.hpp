// Device functions of the dense s-step SGD outer iteration (Algorithm 1 with
// L2 decay) for gfx950. Used both by the one-launch-per-phase kernels and by
// the persistent fused kernel.
#pragma once

#include "common.hpp"

namespace casgd {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;   // Gram tile edge in sampled rows
constexpr int kLPR = 4;     // lanes per row in the update / margin passes
constexpr int kEPL = 4;     // stored elements per lane and row in those passes
constexpr int kNT = 256;    // threads per workgroup of the dense kernels
constexpr int kNW = kNT / 64;

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
    int gt;                 // Gram tiles enumerated (see tile_of)
    int bt;                 // b / kTile when b is a multiple of kTile, else 0
    int gna;                // Gram unit height in 16-row sub-tiles: 4 (64 rows) or 2 (32 rows)
    int ksplit;             // K splits per unit (1, 2, 4 or 8)
    int64_t kchunk;         // K elements per split (multiple of the K step)
    int nslices;            // column slices of the update / margin passes
    int64_t ldy;            // row stride (elements) of the gathered rows: n rounded up to 128
    unsigned* flags;        // FLAG_* words
    unsigned* tile_cnt;     // split-K arrival counters, one per Gram unit (2 * ntiles words)
    float* G[2];            // sb x ldg, row-major, strict block-lower part used
    int64_t ldg;            // row stride of G (sb plus a pad that spreads rows over channels)
    float* Gpart;           // split-K partial units (ntiles * ksplit * 4096 floats)
    float* rp[2];           // nslices x sb partial margins
    float* c;               // sb corrected residual weights
    float* r;               // sb reduced margins (row scales applied)
    unsigned long long* pub; // tagged words exchanged by the recurrence workgroups
    void* Y[3];             // gathered rows of outer iteration h in slot h % 3 (sb x ldy)
    float* yI[3];           // their labels
    float* sI[3];           // their row scales (1 when X has none)
    float* x_hist;          // snapshots or nullptr
    int64_t* t_hist;        // snapshot clocks or nullptr
    int64_t* ptrace;        // phase clock (8 words per outer iteration) or nullptr
    int64_t ptrace_outer;   // outer iterations traced
    int64_t snap_every;
    // fused-launch schedule
    uint64_t h0;            // first outer iteration
    int64_t H;              // outer iterations
    int variant;            // 1 redundant recurrence, 2 single recurrence group
    int gsize;              // workgroups running this problem
    int recur64;            // FP64 recurrence
    int tpr;                // threads per row of the recurrence
    int loss;               // LOSS_* (residual formula of the recurrence)
    int e2e;                // E2E_* end-to-end low-precision emulation
    int g128;               // Gram units are 128 x 128 LDS tiles (gram_tile128)
    int t128;               // lower-triangular 128-tiles enumerated
    // stand-alone 128-tile Gram split along K (gram_tile128_piece), or null
    unsigned long long* sk_slots; // sk_nslots partial slots of kBig * kBig words
    unsigned* sk_epoch;     // the launch tag, advanced before every such launch
    int sk_nslots;          // 0: no K split
};

// The residual formula and the end-to-end rounding mode of a problem. GEN =
// false compiles the default (logistic, no rounding) as constants: the fused
// kernels for that case then carry no run-time branch on them in the chain.
template <bool GEN>
__device__ __forceinline__ int loss_mode(const Dense& P) { return GEN ? P.loss : LOSS_LOGISTIC; }
template <bool GEN>
__device__ __forceinline__ int e2e_mode(const Dense& P) { return GEN ? P.e2e : E2E_OFF; }

__device__ __forceinline__ int slot_of(uint64_t h) { return (int)(h % 3ull); }
inline int slot_of_host(uint64_t h) { return (int)(h % 3ull); }

// Buffer selection by explicit selects: indexing the by-value kernel argument
// with a run-time index would force the whole struct into scratch memory.
template <typename T>
__device__ __forceinline__ T pick3(const T (&a)[3], int k) {
    return k == 0 ? a[0] : (k == 1 ? a[1] : a[2]);
}
template <typename T>
__device__ __forceinline__ T pick2(const T (&a)[2], int k) {
    return k == 0 ? a[0] : a[1];
}

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

// Column-slice width of the update / margin passes: kLPR lanes of kEPL
// elements (16 columns for every storage type, so a narrower type gets as
// many slices -- workgroups -- as FP32; its loads are 8 or 4 bytes).
template <int DT>
constexpr int slice_width() { return kLPR * kEPL; }

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

// Enumerated Gram tile t -> tile coordinates. When b is a multiple of kTile
// (bt = b / kTile tiles per block) only the tiles of the strict block-lower
// triangle are enumerated: block pair q of that triangle (row-major) holds
// tiles q*bt^2 .. (q+1)*bt^2 - 1. Otherwise every lower-triangular tile is
// enumerated and the ones without strict block-lower entries are skipped.
__device__ __forceinline__ bool tile_of(const Dense& P, int t, int& TJ, int& TI) {
    if (P.bt > 0) {
        const int bt2 = P.bt * P.bt;
        const int q = t / bt2, r = t - q * bt2;
        int J, I;
        tile_coords(q, J, I);
        TJ = (J + 1) * P.bt + r / P.bt;
        TI = I * P.bt + r % P.bt;
        return true;
    }
    tile_coords(t, TJ, TI);
    return tile_needed(P, TJ, TI);
}

// MFMA instructions per 16-byte operand vector: FP32 4 (16x16x4), BF16/FP16 1
// (16x16x32), FP8 2 (16x16x32 on 8 bytes each).
template <int DT>
constexpr int mfma_per_vec() { return DT == DT_F32 ? 4 : (DT == DT_FP8 ? 2 : 1); }

// The q-th MFMA of a 16-byte operand pair: acc += A_q B_q^T on a 16x16 tile.
template <int DT>
__device__ __forceinline__ void mfma_q(const V16& a, const V16& b, int q, v4f& acc) {
    if constexpr (DT == DT_F32) {
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(__uint_as_float(a.w[q]), __uint_as_float(b.w[q]),
                                                   acc, 0, 0, 0);
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
        const long av = (long)(((uint64_t)a.w[2 * q + 1] << 32) | a.w[2 * q]);
        const long bv = (long)(((uint64_t)b.w[2 * q + 1] << 32) | b.w[2 * q]);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, bv, acc, 0, 0, 0);
    }
}

// Gather the s*b sampled rows of outer iteration h (Algorithm 1, sampling
// and gather steps) into slot h % 3: row t of Y is X[idx_t, :], zero-padded
// to ldy elements, with its label and row scale; rows sb .. up to the next
// multiple of kTile are zero. One wave copies one row; every lane keeps up
// to eight 16-byte loads in flight.
template <int DT>
__device__ __forceinline__ void gather_rows(const Dense& P, uint64_t h, int wave_id, int nwaves) {
    using T = typename Store<DT>::T;
    constexpr int VEC = Store<DT>::kVec;
    constexpr int U = 8;
    const int slot = slot_of(h);
    T* Y = static_cast<T*>(pick3(P.Y, slot));
    const T* X = static_cast<const T*>(P.X);
    const int lane = threadIdx.x & 63;
    const int64_t nv = P.ldy / VEC;
    const uint64_t t0 = h * (uint64_t)P.sb;
    const V16 zero = {{0u, 0u, 0u, 0u}};
    const int sbpad = (P.sb + 127) / 128 * 128;   // whole 128-row tiles
    for (int t = wave_id; t < sbpad; t += nwaves) {
        T* dst = Y + (int64_t)t * P.ldy;
        if (t >= P.sb) {  // padding rows of the last Gram tile: zeros
            for (int64_t v = lane; v < nv; v += 64)
                *reinterpret_cast<uint4*>(dst + v * VEC) = make_uint4(0u, 0u, 0u, 0u);
            continue;
        }
        const int64_t row = sample_row(P.seed, t0 + t, P.m);
        const T* src = X + row * P.ld;
        for (int64_t v0 = lane; v0 < nv; v0 += 64 * U) {
            V16 buf[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t v = v0 + 64 * u;
                buf[u] = v < nv ? load_v16<DT>(src, v * VEC, P.n) : zero;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t v = v0 + 64 * u;
                if (v < nv)
                    *reinterpret_cast<uint4*>(dst + v * VEC) =
                        make_uint4(buf[u].w[0], buf[u].w[1], buf[u].w[2], buf[u].w[3]);
            }
        }
        if (lane == 0) {
            pick3(P.yI, slot)[t] = P.y ? P.y[row] : 0.0f;
            pick3(P.sI, slot)[t] = P.scale ? P.scale[row] : 1.0f;
        }
    }
}

// LDS of the Gram phase: the cross-wave reduction buffer (4 waves x 4
// sub-tiles x 64 lanes x 16 bytes) and one flag word.
constexpr size_t kGramLds = 4 * 4 * 64 * 16 + 16;

// One Gram work unit: NA*16 rows x 64 columns of the strict block-lower part
// of G (NA = 4: a whole 64x64 tile; NA = 2: the upper or lower half of one,
// half = 0 or 1) over K split `split`, computed by the whole workgroup.
// The four waves split the unit's K range four ways; each computes the whole
// unit as NA x 4 MFMA 16x16 sub-tiles with operands loaded from the gathered
// rows straight into registers (both operands of Y Y^T are K-contiguous
// rows, so no LDS transpose is needed; lane l owns row l%16 of a sub-tile and
// the 16-byte K segment l/16, and any permutation of k that is the same for
// both operands leaves the products unchanged). The waves then reduce
// through LDS in wave order, and wave w keeps sub-tile column w. With more
// than one split, the last workgroup to finish a unit adds the splits'
// partials in split order. Rows are zero-padded to ldy and to a multiple of
// kTile, so no load is guarded.
template <int DT, int NA, bool GEN = true>
__device__ __forceinline__ void gram_unit(const Dense& P, float* Gout, uint64_t h, int unit,
                                          int split, unsigned char* lds) {
    using T = typename Store<DT>::T;
    constexpr int VEC = Store<DT>::kVec;
    constexpr int KSTEP = 4 * VEC;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = NA == 4 ? unit : unit >> 1;
    const int half = NA == 4 ? 0 : unit & 1;
    int TJ, TI;
    if (!tile_of(P, tile, TJ, TI)) return;   // the same for the whole workgroup
    const int row0 = TJ * kTile + half * 32;
    const int li = lane & 15, lg = lane >> 4;
    const int slot = slot_of(h);
    const T* Y = static_cast<const T*>(pick3(P.Y, slot));

    const T* ra[NA];
    const T* rb[4];
#pragma unroll
    for (int a = 0; a < NA; ++a) ra[a] = Y + (int64_t)(row0 + 16 * a + li) * P.ldy + VEC * lg;
#pragma unroll
    for (int c = 0; c < 4; ++c) rb[c] = Y + (int64_t)(TI * kTile + 16 * c + li) * P.ldy + VEC * lg;

    // K range of this wave: a quarter of the split's range, in whole K steps
    const int64_t kpad = (P.n + KSTEP - 1) / KSTEP * KSTEP;
    const int64_t s0 = (int64_t)split * P.kchunk;
    const int64_t s1 = min(kpad, s0 + P.kchunk);
    const int64_t kq = ((s1 - s0 + 3) / 4 + KSTEP - 1) / KSTEP * KSTEP;
    const int64_t k0 = s0 + w * kq;
    const int64_t k1 = min(s1, k0 + kq);

    v4f acc[NA][4];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = v4f{0.f, 0.f, 0.f, 0.f};

    auto ld16 = [&](const T* p, int64_t k) -> V16 {
        const u32x4 q = *reinterpret_cast<const u32x4*>(p + k);
        V16 r;
        r.w[0] = q[0]; r.w[1] = q[1]; r.w[2] = q[2]; r.w[3] = q[3];
        return r;
    };
    // Three operand buffers: the loads of steps k+1 and k+2 are in flight
    // while the MFMAs of step k run. Every load is unconditional (positions
    // past the end are clamped to the last step and not used): a conditional
    // load would become a branch whose join waits for it.
    V16 A0[NA], B0[4], A1[NA], B1[4], A2[NA], B2[4];
    auto load = [&](V16 (&Av)[NA], V16 (&Bv)[4], int64_t k) {
        const int64_t kk = k < k1 ? k : k1 - KSTEP;
#pragma unroll
        for (int a = 0; a < NA; ++a) Av[a] = ld16(ra[a], kk);
#pragma unroll
        for (int c = 0; c < 4; ++c) Bv[c] = ld16(rb[c], kk);
    };
    auto mma = [&](const V16 (&Av)[NA], const V16 (&Bv)[4]) {
        // q outermost: NA*4 independent accumulators between dependent MFMAs
#pragma unroll
        for (int q = 0; q < mfma_per_vec<DT>(); ++q)
#pragma unroll
            for (int a = 0; a < NA; ++a)
#pragma unroll
                for (int c = 0; c < 4; ++c) mfma_q<DT>(Av[a], Bv[c], q, acc[a][c]);
    };
    // Triples of K steps with a single loop exit (a second exit would make the
    // compiler move the accumulators out of and back into AGPRs every step).
    if (k0 < k1) {
        int64_t k = k0;
        load(A0, B0, k0);
        load(A1, B1, k0 + KSTEP);
#pragma unroll 1
        for (; k + 3 * KSTEP <= k1; k += 3 * KSTEP) {
            load(A2, B2, k + 2 * KSTEP);
            mma(A0, B0);
            load(A0, B0, k + 3 * KSTEP);
            mma(A1, B1);
            load(A1, B1, k + 4 * KSTEP);
            mma(A2, B2);
        }
        // 0, 1 or 2 steps remain: A0 holds step k, A1 step k + KSTEP
        if (k < k1) mma(A0, B0);
        if (k + KSTEP < k1) mma(A1, B1);
    }

    // Cross-wave reduction, one sub-tile row at a time: wave w sums sub-tile
    // (a, w) over the four waves in wave order.
    v4f* red = reinterpret_cast<v4f*>(lds);
    v4f part[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) {
#pragma unroll
        for (int c = 0; c < 4; ++c) red[(w * 4 + c) * 64 + lane] = acc[a][c];
        __syncthreads();
        part[a] = red[(0 * 4 + w) * 64 + lane] + red[(1 * 4 + w) * 64 + lane];
        part[a] += red[(2 * 4 + w) * 64 + lane];
        part[a] += red[(3 * 4 + w) * 64 + lane];
        __syncthreads();
    }

    if (P.ksplit > 1) {
        // Publish this split; the last workgroup of the unit adds all splits.
        const int S = P.ksplit;
        v4f* gp = reinterpret_cast<v4f*>(P.Gpart);
        const int64_t ubase = (int64_t)unit * S;
#pragma unroll
        for (int a = 0; a < NA; ++a) gp[(((ubase + split) * 4 + w) * NA + a) * 64 + lane] = part[a];
        // one release (thread 0, after the workgroup barrier) publishes the
        // whole workgroup's partial; the last arrival acquires once
        __syncthreads();
        unsigned* flag = reinterpret_cast<unsigned*>(lds + kGramLds - 16);
        if (threadIdx.x == 0) {
            const unsigned prev = __hip_atomic_fetch_add(P.tile_cnt + unit, 1u, __ATOMIC_RELEASE,
                                                         __HIP_MEMORY_SCOPE_AGENT);
            if (prev == (unsigned)S - 1u) fence_acquire_agent();
            *flag = prev;
        }
        __syncthreads();
        const unsigned prev = *flag;
        __syncthreads();
        if (prev != (unsigned)S - 1u) return;
        // every split's partial of this wave's sub-tiles at once, then the sum
        // in split order
        v4f pv[8][NA];
#pragma unroll
        for (int sp = 0; sp < 8; ++sp)
#pragma unroll
            for (int a = 0; a < NA; ++a)
                if (sp < S)
                    pv[sp][a] = __builtin_nontemporal_load(
                        gp + (((ubase + sp) * 4 + w) * NA + a) * 64 + lane);
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            part[a] = pv[0][a];
#pragma unroll
            for (int sp = 1; sp < 8; ++sp)
                if (sp < S) part[a] += pv[sp][a];
        }
        if (threadIdx.x == 0) atomic_store_relaxed(P.tile_cnt + unit, 0u);
    }

    // Store sub-tiles (a, w): with the 16x16 MFMA output layout, lane l and
    // register v hold row 4*(l/16)+v and column l%16 of a sub-tile. Only
    // strict block-lower entries inside sb x sb are stored; row scales (if
    // any) are applied here.
    const float* sI = pick3(P.sI, slot);
    const int u = TI * kTile + 16 * w + li;
    const float sc = (P.scale && u < P.sb) ? sI[u] : 1.0f;
    const int bu = u / P.b;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int t = row0 + 16 * a + 4 * lg + v;
            if (t < P.sb && u < P.sb && bu < t / P.b) {
                const float sr = P.scale ? sI[t] : 1.0f;
                Gout[(int64_t)t * P.ldg + u] = e2e_round(part[a][v] * sr * sc, e2e_mode<GEN>(P));
            }
        }
    }
}

// ------------------------------------------- Gram, 128 x 128 LDS tiles
// A work unit of this kind is one 128 x 128 tile of the lower triangle of
// G (on the 128 grid) over the whole K range, computed by the workgroup's
// four waves as 2 x 2 quadrants of 64 x 64 (4 x 4 MFMA 16 x 16 tiles each).
// Both row panels (128 rows x 128 bytes of K per chunk) are staged through
// LDS, so every operand byte read from L2 feeds 128 rows of the tile (twice
// the reuse of a 64-row unit whose waves read their operands directly). A
// single LDS buffer with register prefetch: the global loads of chunk c+1
// are issued before the MFMAs of chunk c and written to LDS after them;
// barriers order LDS only, so the loads stay in flight across them. Rows
// are zero-padded to a multiple of 128 and to whole chunks of K.
// LDS layout: row r of a panel at r * 128 bytes, its 16-byte K segment k at
// slot k ^ swz(r). The operand reads (16 consecutive rows, one segment) and
// the staging writes (two rows, all eight segments) then touch 16 distinct
// 16-byte bank groups, with 64 banks and with 32.
constexpr int kBig = 128;                  // tile edge
constexpr int kChunkB = 128;               // bytes of K per row per chunk
constexpr int kRowB = kChunkB;             // LDS row pitch
constexpr size_t kGram128Lds = 2 * (size_t)kBig * kRowB;

__device__ __forceinline__ int swz128(int r) { return ((r >> 1) & 7) ^ ((r & 1) << 2); }

__host__ __device__ inline int tiles128_per_side(int sb) { return (sb + kBig - 1) / kBig; }

// False when the 128-tile (TJ, TI) holds no strict block-lower entry.
__device__ __forceinline__ bool tile128_needed(const Dense& P, int TJ, int TI) {
    const int rlast = min(TJ * kBig + kBig - 1, P.sb - 1);
    return (TI * kBig) / P.b < rlast / P.b;
}

// Position L of the lower-triangular 128-tiles (NT per side) in an order
// that takes them 8 x 8 at a time (super-tiles row by row, the diagonal
// super-tile as a triangle): 64 consecutive tiles then read 16 row panels
// instead of up to 65.
__device__ __forceinline__ void grouped_tile128(int L, int NT, int& TJ, int& TI) {
    constexpr int S = 8;
    int acc = 0;
    for (int SJ = 0; SJ * S < NT; ++SJ) {
        const int rows = min(S, NT - SJ * S);
        for (int SI = 0; SI <= SJ; ++SI) {
            const int cnt = SI < SJ ? rows * S : rows * (rows + 1) / 2;
            if (L < acc + cnt) {
                const int l = L - acc;
                if (SI < SJ) {
                    TJ = SJ * S + l / S;
                    TI = SI * S + l % S;
                } else {
                    tile_coords(l, TJ, TI);
                    TJ += SJ * S;
                    TI += SI * S;
                }
                return;
            }
            acc += cnt;
        }
    }
    TJ = TI = 0;   // not reached for L < NT (NT + 1) / 2
}

template <int DT, bool GEN = true>
__device__ __forceinline__ void gram_tile128_at(const Dense& P, float* Gout, uint64_t h, int TJ,
                                                int TI, unsigned char* lds);

// Lower-triangular 128-tile p in row order.
template <int DT, bool GEN = true>
__device__ __forceinline__ void gram_tile128(const Dense& P, float* Gout, uint64_t h, int tile,
                                             unsigned char* lds) {
    int TJ, TI;
    tile_coords(tile, TJ, TI);
    gram_tile128_at<DT, GEN>(P, Gout, h, TJ, TI, lds);
}

// acc = the products of the tile's row panels over K chunks [c0, c1) of
// 128 bytes (c0 < c1). Lane l of wave w holds, in acc[a][b][v], row
// TJ*128 + (w/2)*64 + 16a + 4(l/16) + v, column TI*128 + (w%2)*64 + 16b + l%16.
template <int DT>
__device__ __forceinline__ void gram128_acc(const Dense& P, uint64_t h, int TJ, int TI, int c0,
                                            int c1, unsigned char* lds, v4f (&acc)[4][4]) {
    using T = typename Store<DT>::T;
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wy = w >> 1, wx = w & 1;
    const unsigned char* Yb = static_cast<const unsigned char*>(pick3(P.Y, slot_of(h)));
    const int64_t ldb = P.ldy * (int64_t)sizeof(T);
    unsigned char* As = lds;
    unsigned char* Bs = lds + (size_t)kBig * kRowB;
    // global -> LDS assignment: 1024 16-byte pieces per panel and chunk,
    // piece v = tid + 256 i: row v / 8, segment v % 8
    const unsigned char* ga[4];
    const unsigned char* gb[4];
    int lo[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int v = tid + 256 * i, row = v >> 3, seg = v & 7;
        ga[i] = Yb + (int64_t)(TJ * kBig + row) * ldb + seg * 16;
        gb[i] = Yb + (int64_t)(TI * kBig + row) * ldb + seg * 16;
        lo[i] = row * kRowB + (seg ^ swz128(row)) * 16;
    }
    // two register sets: the loads of chunk c+2 are issued before the MFMAs
    // of chunk c (two chunks of MFMA work cover the L2 latency); every load
    // is unconditional (past the end it re-reads the last chunk, unused)
    u32x4 ra0[4], rb0[4], ra1[4], rb1[4];
    auto gload = [&](u32x4 (&ra)[4], u32x4 (&rb)[4], int c) {
        const int64_t off = (int64_t)(c < c1 ? c : c1 - 1) * kChunkB;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            ra[i] = *reinterpret_cast<const u32x4*>(ga[i] + off);
            rb[i] = *reinterpret_cast<const u32x4*>(gb[i] + off);
        }
    };
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[a][c] = v4f{0.f, 0.f, 0.f, 0.f};
    const int ar = (wy * 64 + (lane & 15)) * kRowB, br = (wx * 64 + (lane & 15)) * kRowB;
    auto stage = [&](const u32x4 (&ra)[4], const u32x4 (&rb)[4]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            *reinterpret_cast<u32x4*>(As + lo[i]) = ra[i];
            *reinterpret_cast<u32x4*>(Bs + lo[i]) = rb[i];
        }
    };
    // every row this lane reads is (lane & 15) modulo 16: one swizzle
    const int sw = swz128(lane & 15);
    auto compute = [&]() {
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            const int so = (((lane >> 4) + 4 * half) ^ sw) * 16;
            V16 av[4], bv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const u32x4 q = *reinterpret_cast<const u32x4*>(As + ar + a * 16 * kRowB + so);
                av[a].w[0] = q[0]; av[a].w[1] = q[1]; av[a].w[2] = q[2]; av[a].w[3] = q[3];
            }
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const u32x4 q = *reinterpret_cast<const u32x4*>(Bs + br + b * 16 * kRowB + so);
                bv[b].w[0] = q[0]; bv[b].w[1] = q[1]; bv[b].w[2] = q[2]; bv[b].w[3] = q[3];
            }
#pragma unroll
            for (int q = 0; q < mfma_per_vec<DT>(); ++q)
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) mfma_q<DT>(av[a], bv[b], q, acc[a][b]);
        }
    };
    gload(ra0, rb0, c0);
    gload(ra1, rb1, c0 + 1);
#pragma unroll 1
    for (int c = c0; c < c1; c += 2) {
        stage(ra0, rb0);
        lds_barrier();
        gload(ra0, rb0, c + 2);
        compute();
        lds_barrier();
        if (c + 1 < c1) {   // the same for the whole workgroup
            stage(ra1, rb1);
            lds_barrier();
            gload(ra1, rb1, c + 3);
            compute();
            lds_barrier();
        }
    }
}

// Entry (t, u) of the tile with value g: written when it is a strict
// block-lower entry inside sb x sb, with the row scales applied.
template <bool GEN>
__device__ __forceinline__ void gram128_put(const Dense& P, float* Gout, const float* sI, int t,
                                            int u, float g) {
    if (t < P.sb && u < P.sb && u / P.b < t / P.b) {
        const float sr = P.scale ? sI[t] : 1.0f;
        const float sc = P.scale ? sI[u] : 1.0f;
        Gout[(int64_t)t * P.ldg + u] = e2e_round(g * sr * sc, e2e_mode<GEN>(P));
    }
}

template <int DT, bool GEN>
__device__ __forceinline__ void gram_tile128_at(const Dense& P, float* Gout, uint64_t h, int TJ,
                                                int TI, unsigned char* lds) {
    using T = typename Store<DT>::T;
    if (!tile128_needed(P, TJ, TI)) return;   // the same for the whole workgroup
    const int nch = (int)((P.n * (int64_t)sizeof(T) + kChunkB - 1) / kChunkB);
    v4f acc[4][4];
    gram128_acc<DT>(P, h, TJ, TI, 0, nch, lds, acc);
    // store: lane l, register v hold row 4 (l / 16) + v, column l % 16 of a
    // 16 x 16 tile
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wy = w >> 1, wx = w & 1, li = lane & 15, lg = lane >> 4;
    const float* sI = pick3(P.sI, slot_of(h));
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                gram128_put<GEN>(P, Gout, sI, TJ * kBig + wy * 64 + 16 * a + 4 * lg + v,
                                 TI * kBig + wx * 64 + 16 * b + li, acc[a][b][v]);
}

// ------------------------------------ Gram, 128 x 128 tiles split along K
// For Gram matrices with fewer 128-tiles than the device holds workgroups,
// each tile is split into S pieces of consecutive K chunks, one workgroup
// each (all resident: a cooperative launch). Every piece writes its 128 x 128
// partial sums as tagged 64-bit words (value bits low, the launch's tag high,
// single-copy-atomic relaxed accesses: no fence or cache write-back), then
// reduces 1/S of the tile's entries: for each it waits for the S partials
// and adds them in piece order, so the result does not depend on timing.
// Slot q of a tile holds word k * 256 + tid for value k (0..63) of thread
// tid of piece q.
constexpr int kGramSkWords = kBig * kBig;   // 64-bit words per partial

__device__ __forceinline__ void sk_put(unsigned long long* p, unsigned tag, float v) {
    __hip_atomic_store(p, ((unsigned long long)tag << 32) | __float_as_uint(v), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded wait for the tagged value at p; false (timeout flag raised, or
// another workgroup timed out) when it does not arrive.
__device__ __forceinline__ bool sk_wait(const unsigned long long* p, unsigned tag, float& v,
                                        unsigned* flags, unsigned long long spin) {
    unsigned long long n = 0;
    for (;;) {
        const unsigned long long x = __hip_atomic_load(const_cast<unsigned long long*>(p),
                                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((unsigned)(x >> 32) == tag) {
            v = __uint_as_float((unsigned)x);
            return true;
        }
        if (++n > spin) {
            raise_flag(flags, FLAG_TIMEOUT);
            return false;
        }
        if ((n & 63ull) == 0 && atomic_load_relaxed(flags + FLAG_TIMEOUT)) return false;
        __builtin_amdgcn_s_sleep(1);
    }
}

// Piece p of S (1 < S <= 16, S <= the tile's K chunks) of tile (TJ, TI);
// `slots` = the tile's S partial slots.
template <int DT, bool GEN = true>
__device__ __forceinline__ void gram_tile128_piece(const Dense& P, float* Gout, uint64_t h, int TJ,
                                                   int TI, int p, int S, unsigned long long* slots,
                                                   unsigned tag, unsigned long long spin,
                                                   unsigned char* lds) {
    using T = typename Store<DT>::T;
    if (!tile128_needed(P, TJ, TI)) return;   // the same for all pieces
    const int nch = (int)((P.n * (int64_t)sizeof(T) + kChunkB - 1) / kChunkB);
    const int c0 = (int)((int64_t)p * nch / S), c1 = (int)((int64_t)(p + 1) * nch / S);
    v4f acc[4][4];
    gram128_acc<DT>(P, h, TJ, TI, c0, c1, lds, acc);
    const int tid = threadIdx.x;
    unsigned long long* mine = slots + (size_t)p * kGramSkWords + tid;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) sk_put(mine + ((a * 4 + b) * 4 + v) * 256, tag, acc[a][b][v]);
    // this piece's share of the entries: values k0 .. k1-1 of every thread
    const int lane = tid & 63, w = tid >> 6;
    const int wy = w >> 1, wx = w & 1, li = lane & 15, lg = lane >> 4;
    const float* sI = pick3(P.sI, slot_of(h));
    const int k0 = p * 64 / S, k1 = (p + 1) * 64 / S;
    // rounds of KB values: the KB * S words of a round are loaded at once
    // (up to 16 in flight), then checked; a word not there yet is polled
    const int KB = 16 / S;
    bool ok = true;
    for (int kb = k0; kb < k1 && ok; kb += KB) {
        unsigned long long wv[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int kk = i / S, q = i - kk * S;
            if (kk < KB && kb + kk < k1)
                wv[i] = __hip_atomic_load(slots + (size_t)q * kGramSkWords + (kb + kk) * 256 + tid,
                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        float g = 0.f;   // piece sums of one value, added in piece order
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int kk = i / S, q = i - kk * S, k = kb + kk;
            if (ok && kk < KB && k < k1) {
                float v;
                if ((unsigned)(wv[i] >> 32) == tag) {
                    v = __uint_as_float((unsigned)wv[i]);
                } else if (!sk_wait(slots + (size_t)q * kGramSkWords + k * 256 + tid, tag, v,
                                    P.flags, spin)) {
                    ok = false;
                    continue;
                }
                g += v;
                if (q == S - 1) {
                    const int a = k >> 4, b = (k >> 2) & 3, r = k & 3;
                    gram128_put<GEN>(P, Gout, sI, TJ * kBig + wy * 64 + 16 * a + 4 * lg + r,
                                     TI * kBig + wx * 64 + 16 * b + li, g);
                    g = 0.f;
                }
            }
        }
    }
}

// The Gram work of one outer iteration for the workgroups lo .. hi-1 of the
// grid (physical indices). Work = units x K splits (units: whole tiles, or
// half tiles when there are fewer tiles than compute units; see gna). With
// at least ksplit workers, worker w takes only split w % ksplit: workgroups
// are dispatched to the eight XCDs round-robin and ksplit divides 8, so each
// XCD reads one K range of the gathered rows. `lds` holds kGramLds bytes.
template <int DT, bool GEN = true>
__device__ __forceinline__ void gram_phase(const Dense& P, float* Gout, uint64_t h, int lo, int hi,
                                           unsigned char* lds) {
    const int w = blockIdx.x;
    const int nw = hi - lo;
    if (P.g128) {
        for (int u = w - lo; u < P.t128; u += nw) gram_tile128<DT, GEN>(P, Gout, h, u, lds);
        return;
    }
    const int S = P.ksplit;
    const int U = P.gna == 4 ? P.gt : 2 * P.gt;
    if (S == 1) {
        // Units in their natural order (the two halves of a tile, then the
        // tiles of one block row) dealt XCD by XCD: the workgroups of XCD x
        // (physical indices x mod 8) take consecutive units, so the operand
        // rows they share are read through one L2. A bijection of the
        // workgroups, so every unit is computed once, by whichever takes it.
        const int x = w & 7;
        int px = 0, fx = lo;
        for (int y = 0; y < 8; ++y) {
            const int fy = lo + (y - (lo & 7) + 8) % 8;
            const int my = fy < hi ? (hi - fy + 7) / 8 : 0;
            if (y < x) px += my;
            if (y == x) fx = fy;
        }
        for (int u = px + (w - fx) / 8; u < U; u += nw) {
            if (P.gna == 4) gram_unit<DT, 4, GEN>(P, Gout, h, u, 0, lds);
            else gram_unit<DT, 2, GEN>(P, Gout, h, u, 0, lds);
        }
        return;
    }
    if (nw >= S) {
        const int c = w % S;
        const int first = lo + ((c - lo % S) + S) % S;
        const int members = (hi - first + S - 1) / S;
        for (int u = (w - first) / S; u < U; u += members) {
            if (P.gna == 4) gram_unit<DT, 4, GEN>(P, Gout, h, u, c, lds);
            else gram_unit<DT, 2, GEN>(P, Gout, h, u, c, lds);
        }
    } else {
        for (int g = w - lo; g < U * S; g += nw) {
            if (P.gna == 4) gram_unit<DT, 4, GEN>(P, Gout, h, g / S, g % S, lds);
            else gram_unit<DT, 2, GEN>(P, Gout, h, g / S, g % S, lds);
        }
    }
}

// The Gram work of one outer iteration with dynamic shares (no K split):
// every workgroup that reaches it claims whole units from the counter `ctr`
// until none is left, so workgroups that join late (the recurrence
// workgroups, once their chain is done) take what remains. Each unit is
// computed whole by its workgroup: the result does not depend on who
// computed what. `lds` holds kGramLds bytes.
template <int DT, bool GEN = true>
__device__ __forceinline__ void gram_claim(const Dense& P, float* Gout, uint64_t h, unsigned* ctr,
                                           unsigned char* lds) {
    __shared__ unsigned s_unit;
    const unsigned total = (unsigned)(P.g128 ? P.t128 : (P.gna == 4 ? P.gt : 2 * P.gt));
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0)
            s_unit = __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const unsigned u = s_unit;
        if (u >= total) break;
        if (P.g128) gram_tile128<DT, GEN>(P, Gout, h, (int)u, lds);
        else if (P.gna == 4) gram_unit<DT, 4, GEN>(P, Gout, h, (int)u, 0, lds);
        else gram_unit<DT, 2, GEN>(P, Gout, h, (int)u, 0, lds);
    }
}

// ------------------------------------------------------ update and margin
// Column slice `slice` (slice_width<DT>() columns): optionally
//   x <- beta^s x + alpha * sum_t c_t * scale_t * Y_t[slice]      (outer h)
// and then optionally the partial margins of outer hn on the (new) slice:
//   rp_out[slice][t] = Y_t[slice] . x[slice]   (row scale applied later).
// A row segment is read by kLPR lanes with 16-byte loads from the gathered
// rows; NW waves share the rows and every lane keeps U rows in flight.
// Uses LDS `red` (NW * width floats) and `xs` (width floats).
template <int DT, int NW, bool GEN = true>
__device__ __forceinline__ void update_margin_slice(const Dense& P, int slice, const float* c, uint64_t h,
                                    bool do_update, uint64_t hn, bool do_margin, float* rp_out,
                                    float* red, float* xs, int64_t snap_row) {
    using T = typename Store<DT>::T;
    constexpr int VEC = kEPL;
    constexpr int KW = slice_width<DT>();
    constexpr int RPW = kWave / kLPR;
    constexpr int U = 16;   // rows in flight per lane: 1024 rows per workgroup pass
    constexpr int STRIDE = NW * RPW;
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int sub = lane % kLPR, rg = lane / kLPR;
    const int64_t col0 = (int64_t)slice * KW;
    const int64_t kl = col0 + sub * VEC;
    const int sbpad = P.ts * kTile;   // rows of the gathered block (zero-padded)

    if (do_update) {
        const int slot = slot_of(h);
        const T* Y = static_cast<const T*>(pick3(P.Y, slot)) + kl;
        const float* sI = pick3(P.sI, slot);
        float acc[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] = 0.f;
        for (int t0 = w * RPW + rg; t0 < P.sb; t0 += STRIDE * U) {
            V16 v[U];
            float ct[U];
            // Unconditional loads (a conditional load becomes a branch whose
            // join waits for it): rows past sb are clamped into the zero rows
            // that pad the block to whole tiles (or to its last row) and get
            // the weight 0.
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = t0 + u * STRIDE;
                const int tc = t < sbpad ? t : sbpad - 1;
                const int tw = t < P.sb ? t : P.sb - 1;
                v[u] = load_elems<DT, kEPL>(Y + (int64_t)tc * P.ldy);
                const float cw = c[tw] * sI[tw];
                ct[u] = t < P.sb ? cw : 0.f;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc[e] = fmaf(v16_elem<DT>(v[u], e), ct[u], acc[e]);
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e)
#pragma unroll
            for (int off = kLPR; off < kWave; off <<= 1) acc[e] += shfl_xor(acc[e], off);
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
                const int e2e = e2e_mode<GEN>(P);
                xn = e2e_round(P.beta_s * P.x[k] + P.alpha * e2e_round(g, e2e), e2e);
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
        const T* Y = static_cast<const T*>(pick3(P.Y, slot_of(hn))) + kl;
        float xv[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) xv[e] = xs[sub * VEC + e];
        for (int t0 = w * RPW + rg; t0 < P.sb; t0 += STRIDE * U) {
            V16 v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = t0 + u * STRIDE;
                const int tc = t < sbpad ? t : sbpad - 1;
                v[u] = load_elems<DT, kEPL>(Y + (int64_t)tc * P.ldy);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int t = t0 + u * STRIDE;
                float d = 0.f;
#pragma unroll
                for (int e = 0; e < VEC; ++e) d = fmaf(v16_elem<DT>(v[u], e), xv[e], d);
                d = group_sum<kLPR>(d);
                if (sub == 0 && t < P.sb) rp_out[(int64_t)slice * P.sb + t] = d;
            }
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------- recurrence
// The s residual corrections of one outer iteration (Algorithm 1, inner
// loop) with L2 decay, in precision ACC (the u_c slot), by one workgroup of
// NT threads. TPR threads (a power of two) cooperate on one row of a block.
//   z_t = beta^j r_t + alpha * sum_{i<j} beta^(j-1-i) (G_{t, block i} . delta_i)
//   delta_t = glm_delta(z_t, y_t) (logistic: y_t / (1 + exp(y_t z_t)));
//   c_t = beta^(s-1-j) delta_t
// r_t and y_t come either from the partial margins rp (summed over slices,
// times the row scale) and the gathered labels, or directly from r_in / y_in.
// Writes c (global or LDS) and optionally delta_out. Uses LDS `dl` (sb ACC)
// and `pw` (s+1 ACC). The row prefix G[t, 0:jb) does not depend on earlier
// residuals, so each thread issues its loads in batches of kRB independent
// 16-byte loads before consuming them.
constexpr int kRB = 16;

template <typename ACC, int NT, bool GEN = true>
__device__ __forceinline__ void recurrence(const Dense& P, const float* G, const float* rp,
                                           uint64_t h, const float* r_in, const float* y_in,
                                           float* c, float* delta_out, ACC* dl, ACC* pw, int TPR) {
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
    const int slot = slot_of(h);
    for (int j = 0; j < s; ++j) {
        for (int q0 = 0; q0 < b; q0 += RPP) {
            const int q = q0 + tid / TPR;
            const bool active = q < b;
            const int t = j * b + q;
            ACC rr = 0, acc = 0;
            if (active) {
                if (!r_in) {
                    for (int sl = sub; sl < P.nslices; sl += TPR) rr += (ACC)rp[(int64_t)sl * sb + t];
                    rr = group_sum_rt(rr, TPR);
                }
                const float* grow = G + (int64_t)t * P.ldg;
                if (vec4) {
                    // kBB blocks at a time: a thread owns the 16-byte chunks sub,
                    // sub+TPR, ... of the group and issues their loads together;
                    // each chunk lies in one block i and takes its weight
                    // beta^(j-1-i).
                    const int cpb = b >> 2;                 // chunks per block row
                    const bool pow2 = (cpb & (cpb - 1)) == 0;
                    const int lcpb = 31 - __builtin_clz(cpb);
                    constexpr int kBB = 4;
                    for (int i0 = 0; i0 < j; i0 += kBB) {
                        const int nb = min(kBB, j - i0);
                        const int nc = nb * cpb;            // chunks in this group
                        const float4* g4 = reinterpret_cast<const float4*>(grow + i0 * b);
                        for (int c0 = sub; c0 < nc; c0 += kRB * TPR) {
                            float4 g[kRB];
#pragma unroll
                            for (int k = 0; k < kRB; ++k) {
                                const int cc = c0 + k * TPR;
                                g[k] = cc < nc ? g4[cc] : make_float4(0.f, 0.f, 0.f, 0.f);
                            }
#pragma unroll
                            for (int k = 0; k < kRB; ++k) {
                                const int cc = c0 + k * TPR;
                                if (cc < nc) {
                                    const int ib = pow2 ? (cc >> lcpb) : cc / cpb;
                                    const ACC* d = dl + (i0 * b) + 4 * cc;
                                    const ACC part = (ACC)g[k].x * d[0] + (ACC)g[k].y * d[1] +
                                                     (ACC)g[k].z * d[2] + (ACC)g[k].w * d[3];
                                    acc += pw[j - 1 - (i0 + ib)] * part;
                                }
                            }
                        }
                    }
                } else {
                    for (int i = 0; i < j; ++i) {
                        const float* g = grow + i * b;
                        const ACC* d = dl + i * b;
                        ACC part = 0;
                        for (int p = sub; p < b; p += TPR) part += (ACC)g[p] * d[p];
                        acc += pw[j - 1 - i] * part;
                    }
                }
                acc = group_sum_rt(acc, TPR);
            }
            if (active && sub == 0) {
                ACC r, yv;
                if (r_in) {
                    r = (ACC)r_in[t];
                    yv = (ACC)y_in[t];
                } else {
                    r = e2e_round(rr * (ACC)pick3(P.sI, slot)[t], e2e_mode<GEN>(P));
                    yv = (ACC)pick3(P.yI, slot)[t];
                }
                const int e2e = e2e_mode<GEN>(P);
                const ACC z = e2e_round(pw[j] * r + alpha * e2e_round(acc, e2e), e2e);
                const ACC d = e2e_round(glm_delta<ACC>(z, yv, loss_mode<GEN>(P)), e2e);
                if (!isfinite(z) || !isfinite(d)) raise_flag(P.flags, FLAG_NONFINITE);
                dl[t] = d;
                c[t] = (float)e2e_round(pw[s - 1 - j] * d, e2e);
                if (delta_out) delta_out[t] = (float)d;
            }
        }
        __syncthreads();
    }
}

}  // namespace casgd

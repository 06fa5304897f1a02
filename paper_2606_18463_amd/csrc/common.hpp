// Device-side building blocks shared by the libcasgd kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace casgd {

constexpr int kWave = 64;

// ---------------------------------------------------------------- sampling
// Counter-based SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output t of
// the stream that starts in state `seed` is mix(seed + (t+1) * golden gamma).
// A sample is mapped to a row by the high half of the 128-bit product with m.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t t) {
    uint64_t z = seed + (t + 1ull) * 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ int64_t sample_row(uint64_t seed, uint64_t t, uint64_t m) {
    return (int64_t)__umul64hi(splitmix64(seed, t), m);
}

// ------------------------------------------------------------------ losses
// The three generalized linear models of Sec. 2.1; the residual is
// delta = -dL/dz at the margin z (Sec. 3.1):
//   logistic  L = log(1 + exp(-y z))      delta = y / (1 + exp(y z)) = y (1 - sigma(y z))
//   linear    L = (z - y)^2 / 2           delta = y - z
//   Poisson   L = exp(z) - y z            delta = y - exp(z)
enum : int { LOSS_LOGISTIC = 0, LOSS_LINEAR = 1, LOSS_POISSON = 2 };

template <typename ACC>
__device__ __forceinline__ ACC glm_delta(ACC z, ACC y, int loss) {
    if (loss == LOSS_LINEAR) return y - z;
    if (loss == LOSS_POISSON) return y - exp(z);
    return y / ((ACC)1 + exp(y * z));
}

// ----------------------------------------------------------- storage types
enum : int { DT_F32 = 0, DT_BF16 = 1, DT_F16 = 2, DT_FP8 = 3 };

template <int DT> struct Store;
template <> struct Store<DT_F32> { using T = float;    static constexpr int kVec = 4;  };
template <> struct Store<DT_BF16> { using T = uint16_t; static constexpr int kVec = 8;  };
template <> struct Store<DT_F16> { using T = uint16_t; static constexpr int kVec = 8;  };
template <> struct Store<DT_FP8> { using T = uint8_t;  static constexpr int kVec = 16; };

// OCP E4M3: sign, 4 exponent bits (bias 7), 3 mantissa bits; exponent field 0
// is subnormal (m * 2^-9). Code 0x7f/0xff is NaN and never produced here.
// Decoded by gfx950's FP8 convert (OCP E4M3; every code is checked against the
// oracle's table): byte `sel` of the word w.
template <int SEL>
__device__ __forceinline__ float e4m3_byte(uint32_t w) {
    return __builtin_amdgcn_cvt_f32_fp8((int)w, SEL);
}
__device__ __forceinline__ float e4m3_sel(uint32_t w, int sel) {
    switch (sel & 3) {
        case 0: return e4m3_byte<0>(w);
        case 1: return e4m3_byte<1>(w);
        case 2: return e4m3_byte<2>(w);
        default: return e4m3_byte<3>(w);
    }
}
__device__ __forceinline__ float e4m3_to_float(uint32_t c) { return e4m3_byte<0>(c); }

// Round to nearest, ties to even, saturating to +-448.
__device__ __forceinline__ uint32_t float_to_e4m3(float v) {
    const uint32_t sign = (__float_as_uint(v) >> 24) & 0x80u;
    const float a = fabsf(v);
    if (!(a < 448.0f)) return sign | 0x7eu;            // >= 448 (and NaN) -> 448
    if (a < 0.015625f) {                               // below 2^-6: subnormal grid 2^-9
        const float q = rintf(a * 512.0f);             // exact scaling, RNE
        return sign | (uint32_t)q;                     // q == 8 is the smallest normal
    }
    const uint32_t bits = __float_as_uint(a);
    int e = (int)(bits >> 23) - 127;
    const uint32_t mant = bits & 0x7fffffu;
    uint32_t q = mant >> 20;
    const uint32_t rem = mant & 0xfffffu;
    if (rem > 0x80000u || (rem == 0x80000u && (q & 1u))) ++q;
    if (q == 8u) { q = 0u; ++e; }
    const int ef = e + 7;
    if (ef > 15 || (ef == 15 && q == 7u)) return sign | 0x7eu;
    return sign | ((uint32_t)ef << 3) | q;
}

__device__ __forceinline__ float bf16_to_float(uint32_t h) { return __uint_as_float(h << 16); }

__device__ __forceinline__ uint32_t float_to_bf16(float v) {
    const uint32_t u = __float_as_uint(v);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}

__device__ __forceinline__ float f16_to_float(uint32_t h) {
    _Float16 x;
    uint16_t hb = (uint16_t)h;
    __builtin_memcpy(&x, &hb, 2);
    return (float)x;
}

__device__ __forceinline__ uint32_t float_to_f16(float v) {
    _Float16 x = (_Float16)v;
    uint16_t hb;
    __builtin_memcpy(&hb, &x, 2);
    return hb;
}

// End-to-end low-precision emulation (the paper's all-BF16 and all-FP16
// baselines): every slot's output -- Gram entries, margins, the inner
// correction sums, margins z, residuals, weights c, the gradient and the
// iterate -- is rounded to the format (round to nearest even); sums inside a
// kernel accumulate in FP32.
enum : int { E2E_OFF = 0, E2E_BF16 = 1, E2E_F16 = 2 };
__device__ __forceinline__ float e2e_round(float v, int mode) {
    if (mode == E2E_BF16) return bf16_to_float(float_to_bf16(v));
    if (mode == E2E_F16) return f16_to_float(float_to_f16(v));
    return v;
}
__device__ __forceinline__ double e2e_round(double v, int mode) {
    return mode == E2E_OFF ? v : (double)e2e_round((float)v, mode);
}

// A 16-byte vector of stored elements and its conversion to FP32.
struct V16 { uint32_t w[4]; };

template <int DT>
__device__ __forceinline__ float v16_elem(const V16& v, int e) {
    if constexpr (DT == DT_F32) {
        return __uint_as_float(v.w[e]);
    } else if constexpr (DT == DT_BF16) {
        const uint32_t w = v.w[e >> 1];
        return (e & 1) ? __uint_as_float(w & 0xffff0000u) : __uint_as_float(w << 16);
    } else if constexpr (DT == DT_F16) {
        const uint32_t w = v.w[e >> 1];
        return f16_to_float((e & 1) ? (w >> 16) : (w & 0xffffu));
    } else {
        return e4m3_sel(v.w[e >> 2], e & 3);
    }
}

// Load the EPL stored elements at p (EPL * sizeof(T) bytes, aligned to that
// size) into the first words of a V16 (element e at the same place as in a
// full 16-byte vector, so v16_elem reads it).
template <int DT, int EPL>
__device__ __forceinline__ V16 load_elems(const typename Store<DT>::T* p) {
    using T = typename Store<DT>::T;
    constexpr int BYTES = EPL * (int)sizeof(T);
    static_assert(BYTES == 16 || BYTES == 8 || BYTES == 4, "4, 8 or 16 bytes per load");
    V16 v;
    if constexpr (BYTES == 16) {
        const uint4 q = *reinterpret_cast<const uint4*>(p);
        v.w[0] = q.x; v.w[1] = q.y; v.w[2] = q.z; v.w[3] = q.w;
    } else if constexpr (BYTES == 8) {
        const uint2 q = *reinterpret_cast<const uint2*>(p);
        v.w[0] = q.x; v.w[1] = q.y; v.w[2] = 0u; v.w[3] = 0u;
    } else {
        v.w[0] = *reinterpret_cast<const uint32_t*>(p);
        v.w[1] = v.w[2] = v.w[3] = 0u;
    }
    return v;
}

// Load kVec elements starting at element k of a row with n valid elements.
// Full vectors use one 16-byte load; a vector crossing n is read element-wise
// and padded with zeros; a vector starting at or beyond n is all zeros.
template <int DT>
__device__ __forceinline__ V16 load_v16(const typename Store<DT>::T* row, int64_t k, int64_t n) {
    constexpr int VEC = Store<DT>::kVec;
    V16 v;
    if (k + VEC <= n) {
        const uint4 u = *reinterpret_cast<const uint4*>(row + k);
        v.w[0] = u.x; v.w[1] = u.y; v.w[2] = u.z; v.w[3] = u.w;
        return v;
    }
    v.w[0] = v.w[1] = v.w[2] = v.w[3] = 0u;
    if (k >= n) return v;
    constexpr int BYTES = 16 / VEC;
    for (int e = 0; e < VEC; ++e) {
        if (k + e < n) {
            uint32_t bits;
            if constexpr (BYTES == 4) bits = reinterpret_cast<const uint32_t*>(row)[k + e];
            else if constexpr (BYTES == 2) bits = reinterpret_cast<const uint16_t*>(row)[k + e];
            else bits = reinterpret_cast<const uint8_t*>(row)[k + e];
            v.w[(e * BYTES) >> 2] |= bits << (8 * ((e * BYTES) & 3));
        }
    }
    return v;
}

// ------------------------------------------------------- wave reductions
template <typename T>
__device__ __forceinline__ T shfl_xor(T v, int mask) {
    return __shfl_xor(v, mask, kWave);
}

// Sum over groups of `G` consecutive lanes (G a power of two <= 64); every lane
// of the group receives the total.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int off = 1; off < G; off <<= 1) v += shfl_xor(v, off);
    return v;
}

// ------------------------------------------------- device-scope atomics
__device__ __forceinline__ unsigned atomic_add_acq_rel(unsigned* p, unsigned v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned atomic_load_acquire(unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned atomic_load_relaxed(unsigned* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_store_release(unsigned* p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void fence_acquire_agent() {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}
__device__ __forceinline__ void fence_release_agent() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
}
__device__ __forceinline__ void atomic_store_relaxed(unsigned* p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroup barrier that orders LDS accesses only: global loads issued
// before it (prefetches) stay in flight across it, where __syncthreads()
// would wait for them.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Flag words at the start of every workspace.
enum : int {
    FLAG_NONFINITE = 0,   // set when a margin, residual or weight is NaN/Inf
    FLAG_TIMEOUT = 1,     // set when a grid barrier exceeded its spin limit
    FLAG_BAR_COUNT = 32,  // first barrier word (everything from here is cleared
                          // before a fused launch)
    // a barrier's words from its base: generation, top arrival counter, then
    // eight group counters, each on its own 128-byte line
    BAR_GEN = 0,
    BAR_TOP = 32,
    BAR_GROUP = 64,       // + 32 * group
    BAR_WORDS = 320,
    FLAG_BAR_MAIN = 32,   // the grid barrier
    FLAG_BAR_SUB = 352,   // a barrier among a subset of the workgroups
    FLAG_SLICES = 672,    // update slices finished in this launch (own line)
    FLAG_GRAM_CLAIM = 704,// Gram units claimed in this outer iteration, per parity (own line)
    FLAG_XCD_CENSUS = 736,// workgroups of the fused launch on each XCD (8 words, own line)
    FLAG_SLICE_CENSUS = 768, // update-slice workgroups on each XCD (8 words)
    FLAG_SLICE_XCD = 776, // update slices finished on each XCD in this launch (8 words)
    FLAG_WORDS = 800
};

// The XCD this workgroup runs on (hardware register XCC_ID, bits 3:0).
__device__ __forceinline__ unsigned xcd_id() {
    return (unsigned)__builtin_amdgcn_s_getreg(20 | (3 << 11)) & 7u;
}

// Entry points without a workspace pass flags == nullptr and report nothing.
__device__ __forceinline__ void raise_flag(unsigned* flags, int which) {
    if (flags) __hip_atomic_fetch_or(&flags[which], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier for a launch whose workgroups are all resident (the
// cooperative launch guarantees it). Sense is kept in a generation counter.
// Arrival is hierarchical: member m counts in group m % 8 (one counter per
// group, each on its own cache line), and the last arrival of each group
// counts at the top; the last one there advances the generation. That keeps
// the number of atomics serialised on one address near nblocks / 8 + 8.
// One thread per workgroup synchronises for the whole workgroup (after a
// workgroup barrier, its agent-scope release and acquire cover every wave):
// agent-scope release and acquire write back and invalidate the XCD's L2, so
// they are issued once per workgroup, and the poll itself uses relaxed loads
// (which read the coherent copy without touching the caches).
// The wait is bounded: after `spin_limit` polls the timeout flag is raised
// and the workgroup leaves the kernel; every other one then stops at its
// next wait (which can no longer complete without it, and which checks the
// flag every 256 polls), so a launch can never wait forever. A barrier that
// did complete needs no check of the flag on the way out (one memory round
// trip less per barrier). Returns false when the kernel must stop.
__device__ __forceinline__ bool barrier_at(unsigned* flags, int base, unsigned member,
                                           unsigned nblocks, unsigned long long spin_limit) {
    __shared__ int s_stop;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned ng = nblocks < 8u ? nblocks : 8u;
        const unsigned g = member % ng;
        const unsigned in_group = (nblocks - g + ng - 1) / ng;
        unsigned* gen = flags + base + BAR_GEN;
        unsigned* top = flags + base + BAR_TOP;
        unsigned* cnt = flags + base + BAR_GROUP + 32 * g;
        const unsigned g0 = atomic_load_relaxed(gen);
        int stop = 0;
        bool advanced = false;
        const unsigned a = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (a == in_group - 1) {
            fence_acquire_agent();
            atomic_store_relaxed(cnt, 0u);
            const unsigned t =
                __hip_atomic_fetch_add(top, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (t == ng - 1) {
                atomic_store_relaxed(top, 0u);
                atomic_store_release(gen, g0 + 1u);
                advanced = true;
            }
        }
        if (!advanced) {
            unsigned long long spins = 0;
            while (atomic_load_relaxed(gen) == g0) {
                if (++spins > spin_limit) {
                    raise_flag(flags, FLAG_TIMEOUT);
                    stop = 1;
                    break;
                }
                if ((spins & 255ull) == 0 && atomic_load_relaxed(flags + FLAG_TIMEOUT)) {
                    stop = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            fence_acquire_agent();
        }
        s_stop = stop;
    }
    __syncthreads();
    return s_stop == 0;
}

// Bounded wait (thread 0 for the workgroup) until the counter at word `w`
// reaches `want`, then an acquire: the counted workgroups' writes are
// visible to the whole workgroup. Returns false on timeout.
__device__ __forceinline__ bool wait_count(unsigned* flags, int w, unsigned want,
                                           unsigned long long spin_limit) {
    __shared__ int s_ok;
    if (threadIdx.x == 0) {
        int ok = 1;
        unsigned long long spins = 0;
        while (atomic_load_relaxed(flags + w) < want) {
            if (++spins > spin_limit) {
                raise_flag(flags, FLAG_TIMEOUT);
                ok = 0;
                break;
            }
            if ((spins & 255ull) == 0 && atomic_load_relaxed(flags + FLAG_TIMEOUT)) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        fence_acquire_agent();
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

// The grid barrier: every workgroup of the launch (or of one problem's group).
__device__ __forceinline__ bool grid_barrier(unsigned* flags, unsigned member, unsigned nblocks,
                                             unsigned long long spin_limit) {
    return barrier_at(flags, FLAG_BAR_MAIN, member, nblocks, spin_limit);
}

// Arrival grouped by XCD for a launch whose XCD census is known (xcd_census):
// each wave first waits for its own memory operations, so the workgroup's
// stores have reached its XCD's L2 (the vector L1 is write-through); members
// arrive with a relaxed count, and only the last arrival of each XCD writes
// that L2 back (one agent-scope release per XCD instead of one per
// workgroup, for the stores of every workgroup there). The exit keeps one
// acquire per workgroup. `members`: workgroups of this barrier on this XCD;
// `ngroups`: XCDs that hold any. Same words and bounded wait as barrier_at.
__device__ __forceinline__ bool grid_barrier_xcd(unsigned* flags, unsigned members,
                                                 unsigned ngroups,
                                                 unsigned long long spin_limit) {
    __shared__ int s_stop;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned* gen = flags + FLAG_BAR_MAIN + BAR_GEN;
        unsigned* top = flags + FLAG_BAR_MAIN + BAR_TOP;
        unsigned* cnt = flags + FLAG_BAR_MAIN + BAR_GROUP + 32 * xcd_id();
        const unsigned g0 = atomic_load_relaxed(gen);
        int stop = 0;
        bool advanced = false;
        const unsigned a = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (a == members - 1) {
            fence_release_agent();
            atomic_store_relaxed(cnt, 0u);
            // released just above; only the last arrival at the top acquires
            // (the other XCDs' releases), before releasing the generation
            const unsigned t =
                __hip_atomic_fetch_add(top, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (t == ngroups - 1) {
                fence_acquire_agent();
                atomic_store_relaxed(top, 0u);
                atomic_store_release(gen, g0 + 1u);
                advanced = true;
            }
        }
        if (!advanced) {
            unsigned long long spins = 0;
            while (atomic_load_relaxed(gen) == g0) {
                if (++spins > spin_limit) {
                    raise_flag(flags, FLAG_TIMEOUT);
                    stop = 1;
                    break;
                }
                if ((spins & 255ull) == 0 && atomic_load_relaxed(flags + FLAG_TIMEOUT)) {
                    stop = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            fence_acquire_agent();
        }
        s_stop = stop;
    }
    __syncthreads();
    return s_stop == 0;
}

// Counts this workgroup in the launch's XCD census, and in the census of
// update-slice workgroups when `slice` (before the launch's first grid
// barrier; the census words start at zero).
__device__ __forceinline__ void xcd_census_add(unsigned* flags, bool slice) {
    if (threadIdx.x == 0) {
        const unsigned x = xcd_id();
        __hip_atomic_fetch_add(flags + FLAG_XCD_CENSUS + x, 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        if (slice)
            __hip_atomic_fetch_add(flags + FLAG_SLICE_CENSUS + x, 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Slices finished by this workgroup's XCD are published together: the
// workgroup waits for its own stores (they are in the XCD's L2) and counts
// itself relaxed; the last slice of the XCD in this outer iteration writes
// that L2 back once and adds the XCD's `per_xcd` slices to the count at word
// `w` that the margin reducers wait on.
__device__ __forceinline__ void publish_slice_xcd(unsigned* flags, int w, unsigned per_xcd) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned a = __hip_atomic_fetch_add(flags + FLAG_SLICE_XCD + xcd_id(), 1u,
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((a + 1u) % per_xcd == 0u) {
            fence_release_agent();
            __hip_atomic_fetch_add(flags + w, per_xcd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// After the first grid barrier: workgroups on this XCD and XCDs in use.
__device__ __forceinline__ void xcd_census_read(unsigned* flags, unsigned& members,
                                                unsigned& ngroups, unsigned& slices) {
    const unsigned me = xcd_id();
    members = 0;
    ngroups = 0;
#pragma unroll
    for (unsigned x = 0; x < 8; ++x) {
        const unsigned c = atomic_load_relaxed(flags + FLAG_XCD_CENSUS + x);
        if (c) ++ngroups;
        if (x == me) members = c;
    }
    slices = atomic_load_relaxed(flags + FLAG_SLICE_CENSUS + me);
}

}  // namespace casgd

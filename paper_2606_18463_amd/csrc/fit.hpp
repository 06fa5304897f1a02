// The fused persistent fit: one cooperative launch runs every outer
// iteration, with phases separated by the bounded grid barrier. Included by
// one translation unit per storage type (fit_<type>.hip) and by the batched
// launch.
#pragma once

#include "internal.hpp"
#include "recurrence.hpp"

namespace casgd {

// Phase clock: thread 0 of the workgroup records the device clock in word
// `k` of outer iteration hh when tracing is on.
__device__ __forceinline__ void phase_mark(const Dense& P, int64_t hh, int k) {
    if (P.ptrace && threadIdx.x == 0 && hh < P.ptrace_outer)
        P.ptrace[hh * 8 + k] = (int64_t)wall_clock64();
}

// Column slice handled by slice workgroup wg when every slice workgroup has
// one (nslices <= nb): the slices of one XCD (workgroups x, x + 8, ...) are
// contiguous, so the two 64-byte halves of a 128-byte line of a gathered row
// (neighbouring 16-column slices) are read through the same L2. Partial
// margins stay indexed by slice, so results do not depend on the mapping.
__device__ __forceinline__ int slice_of(int wg, int nslices, int nb) {
    if (nslices > nb || (nslices & 7)) return wg;
    return (wg & 7) * (nslices >> 3) + (wg >> 3);
}

// Lanes that reduce one row's partial margins: 8, 16 or 32, from the slice
// count alone (so a batched problem sums in the same order as a solo one),
// at most four slices per lane from 32 lanes on.
__device__ __forceinline__ int margin_lanes(int nslices) {
    return nslices >= 128 ? 32 : (nslices >= 64 ? 16 : 8);
}

// Margins of outer iteration h from the slices' partial sums: L lanes per
// row (margin_lanes), lane e adding slices e, e+L, ... in order, then a fixed
// tree over the L lanes; times the row scale. Threads gtid of nthreads
// (multiples of 32).
template <bool GEN = true>
__device__ __forceinline__ void reduce_margins(const Dense& P, const float* rp, uint64_t h,
                                               float* r_out, int gtid, int nthreads) {
    const float* sI = pick3(P.sI, slot_of(h));
    const int L = margin_lanes(P.nslices);
    const int e = gtid & (L - 1);
    // the L lanes of a group share t, so they run the loop together
    for (int t = gtid / L; t < P.sb; t += nthreads / L) {
        float a = 0.f;
#pragma unroll 4
        for (int sl = e; sl < P.nslices; sl += L) a += rp[(int64_t)sl * P.sb + t];
        for (int off = 1; off < L; off <<= 1) a += shfl_xor(a, off);
        if (e == 0) r_out[t] = e2e_round(a * sI[t], e2e_mode<GEN>(P));
    }
}

// The recurrence workgroup of rank `rank` (0 = chain, 1.. = helpers) for the
// problem's b (16, 32, 64 or 128).
template <typename ACC, bool GEN = true>
__device__ __forceinline__ void rec_multi_rank(const Dense& P, const float* G, const float* r,
                                               const float* y, float* c, unsigned long long spin,
                                               unsigned char* lds, int rank) {
    switch (P.b) {
        case 16:
            recurrence_multi<ACC, 1, rec_window<1>(), GEN>(P, G, r, y, c, nullptr, P.pub, spin, lds,
                                                          rank);
            break;
        case 32:
            recurrence_multi<ACC, 2, rec_window<2>(), GEN>(P, G, r, y, c, nullptr, P.pub, spin, lds,
                                                          rank);
            break;
        case 64:
            recurrence_multi<ACC, 4, rec_window<4>(), GEN>(P, G, r, y, c, nullptr, P.pub, spin, lds,
                                                          rank);
            break;
        default:
            recurrence_multi<ACC, 8, rec_window<8>(), GEN>(P, G, r, y, c, nullptr, P.pub, spin, lds,
                                                          rank);
            break;
    }
}

// LDS bytes of the persistent kernel: recurrence history, decay powers, the
// workgroup's copy of c (variant 1), and the update's reduction buffers.
__host__ __device__ inline size_t fit_lds_bytes(int sb, int s, int acc_bytes, int kw) {
    size_t off = (size_t)sb * acc_bytes;
    off += (size_t)(s + 1) * acc_bytes;
    off = (off + 15) & ~(size_t)15;
    off += (size_t)sb * 4;                // c copy
    off += (size_t)kNW * kw * 4 + kw * 4; // red + xs
    // the Gram phase reuses the same memory (phases never overlap in a workgroup)
    return s > 1 && off < kGram128Lds ? kGram128Lds : off;
}

// One problem's whole fit on the workgroups wg = 0 .. nb-1 of its group (the
// grid, or one group of a batched launch), with the group's own barrier.
// Per outer iteration h:
//  * variant 3 (MULTI): phase A, workgroups 0 .. R run the multi-workgroup
//    recurrence of h while the others build the Gram of h+1 (claiming units,
//    which the recurrence workgroups join when done); barrier;
//    phase B, the column-slice workgroups apply the update of h fused with
//    the partial margins of h+1, the others gather the rows of h+2 and then
//    reduce those margins once every slice has counted in; barrier.
//  * variant 1: every update workgroup runs the single-workgroup recurrence
//    itself, updates its slices, then everybody builds the next Gram and
//    gathers; one barrier (small s*b, plain SGD).
//  * variant 2: workgroup 0 runs the single-workgroup recurrence while the
//    others build the next Gram and gather; barrier; update; barrier.
template <int DT, typename ACC, bool MULTI, bool GEN = true>
__device__ __forceinline__ void fit_body(const Dense& P, int wg, int nb, unsigned long long spin,
                                         unsigned char* lds) {
    constexpr int KW = slice_width<DT>();
    ACC* dl = reinterpret_cast<ACC*>(lds);
    ACC* pw = dl + P.sb;
    size_t off = (size_t)P.sb * sizeof(ACC) + (size_t)(P.s + 1) * sizeof(ACC);
    off = (off + 15) & ~(size_t)15;
    float* cl = reinterpret_cast<float*>(lds + off);
    float* red = cl + P.sb;
    float* xs = red + kNW * KW;

    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const bool has_gram = P.s > 1;
    // physical workgroup range of this problem (the Gram phase maps K splits
    // to XCDs by physical index)
    const int base = (int)blockIdx.x - wg;
    const uint64_t h0 = P.h0;
    const int64_t H = P.H;
    const int tpr = P.tpr;

    if (threadIdx.x == 0 && wg == 0 && P.t_hist) P.t_hist[0] = (int64_t)wall_clock64();
    const int gw = wg * kNW + wave, ngw = nb * kNW;

    // Prologue: gather the rows of h0 and h0+1; then the Gram of h0 and the
    // margins of h0 from the incoming x.
    // The first barrier also completes the XCD census; every later one
    // writes each XCD's L2 back once (grid_barrier_xcd).
    xcd_census_add(P.flags, wg < P.nslices && nb > P.nslices);
    gather_rows<DT>(P, h0, gw, ngw);
    if (H > 1) gather_rows<DT>(P, h0 + 1, gw, ngw);
    if (!grid_barrier(P.flags, wg, nb, spin)) return;
    unsigned xm, xg, xs_slices;
    xcd_census_read(P.flags, xm, xg, xs_slices);
    if (has_gram) gram_phase<DT, GEN>(P, P.G[0], h0, base, base + nb, lds);
    for (int sl = wg; sl < P.nslices; sl += nb)
        update_margin_slice<DT, kNW, GEN>(P, slice_of(sl, P.nslices, nb), nullptr, 0, false, h0,
                                         true, P.rp[0], red, xs, -1);
    if (!grid_barrier_xcd(P.flags, xm, xg, spin)) return;
    for (int64_t hh = 0; hh < H; ++hh) {
        const uint64_t h = h0 + (uint64_t)hh;
        const int cur = (int)(hh & 1), nxt = cur ^ 1;
        const bool more = hh + 1 < H;
        const bool more2 = hh + 2 < H;
        const bool snap = P.snap_every > 0 && ((hh + 1) % P.snap_every) == 0;
        const int64_t snap_row = snap ? (hh + 1) / P.snap_every - 1 : -1;
        if (MULTI && P.variant == 3) {
            // Phase A: workgroups 0 .. nrec-1 reduce the margins of h, meet
            // at their own barrier and run the recurrence of h (chain +
            // helpers); the others build the Gram of h+1.
            const int nrec = 1 + rec_helpers(P.b, P.s);
            if (wg == 0) phase_mark(P, hh, 0);
            if (hh == 0) {
                // margins of h0 (from the prologue): reduced by the recurrence
                // workgroups themselves
                if (wg < nrec) {
                    reduce_margins<GEN>(P, pick2(P.rp, cur), h, P.r, wg * kNT + (int)threadIdx.x,
                                   nrec * kNT);
                    if (!barrier_at(P.flags, FLAG_BAR_SUB, wg, nrec, spin)) return;
                }
            }
            // With more Gram units than Gram workgroups (and no K split) the
            // units are claimed dynamically, and the recurrence workgroups join
            // once their chain is done; one round of units is dealt statically.
            const int units = P.g128 ? P.t128 : (P.gna == 4 ? P.gt : 2 * P.gt);
            const bool claim = (P.g128 || P.ksplit == 1) && units > nb - nrec;
            if (wg < nrec) {
                rec_multi_rank<ACC, GEN>(P, pick2(P.G, cur), P.r, pick3(P.yI, slot_of(h)), P.c, spin, lds,
                                    wg);
                if (wg == 0) phase_mark(P, hh, 1);
            } else if (has_gram && more && !claim) {
                gram_phase<DT, GEN>(P, pick2(P.G, nxt), h + 1, base + nrec, base + nb, lds);
            }
            if (has_gram && more && claim)
                gram_claim<DT, GEN>(P, pick2(P.G, nxt), h + 1, P.flags + FLAG_GRAM_CLAIM + (hh & 1), lds);
            if (wg == nrec) phase_mark(P, hh, 2);
            if (wg == nb - 1) phase_mark(P, hh, 6);
            if (!grid_barrier_xcd(P.flags, xm, xg, spin)) return;
            if (wg == 0) phase_mark(P, hh, 3);
            // every claim of this outer iteration is done: reset the counter of
            // this parity, next used two outer iterations on
            if (wg == 0 && threadIdx.x == 0)
                atomic_store_relaxed(P.flags + FLAG_GRAM_CLAIM + (hh & 1), 0u);
            // Phase B: update of h fused with the margins of h+1 on the
            // column slices; workgroups without a slice gather the rows of h+2.
            // With more workgroups than slices, the ones without a slice gather
            // the rows of h+2, then wait until every slice has published its
            // partial margins (a counter that grows by nslices per outer
            // iteration) and reduce them, so the next recurrence finds them.
            // Otherwise everybody updates, gathers, and the reduction waits
            // for the next phase.
            const bool split = nb > P.nslices;
            for (int sl = wg; sl < P.nslices; sl += nb)
                update_margin_slice<DT, kNW, GEN>(P, slice_of(sl, P.nslices, nb), P.c, h, true, h + 1,
                                                 more, pick2(P.rp, nxt), red, xs, snap_row);
            if (wg == 0) phase_mark(P, hh, 4);
            if (split && wg < P.nslices && more) publish_slice_xcd(P.flags, FLAG_SLICES, xs_slices);
            if (more2) {
                if (split) {
                    if (wg >= P.nslices)
                        gather_rows<DT>(P, h + 2, gw - P.nslices * kNW, ngw - P.nslices * kNW);
                } else {
                    gather_rows<DT>(P, h + 2, gw, ngw);
                }
            }
            if (split && wg >= P.nslices && more) {
                const unsigned want = (unsigned)P.nslices * (unsigned)(hh + 1);
                if (!wait_count(P.flags, FLAG_SLICES, want, spin)) return;
                reduce_margins<GEN>(P, pick2(P.rp, nxt), h + 1, P.r,
                               (wg - P.nslices) * kNT + (int)threadIdx.x, (nb - P.nslices) * kNT);
            }
            if (wg == nb - 1) phase_mark(P, hh, 7);
            if (!grid_barrier_xcd(P.flags, xm, xg, spin)) return;
            if (wg == 0) phase_mark(P, hh, 5);
            if (!split && more) {
                if (wg < nrec) {
                    reduce_margins<GEN>(P, pick2(P.rp, nxt), h + 1, P.r, wg * kNT + (int)threadIdx.x,
                                   nrec * kNT);
                    if (!barrier_at(P.flags, FLAG_BAR_SUB, wg, nrec, spin)) return;
                }
            }
        } else if (P.variant == 1) {
            if (wg < P.nslices) {
                recurrence<ACC, kNT, GEN>(P, pick2(P.G, cur), pick2(P.rp, cur), h, nullptr, nullptr, cl,
                                     nullptr, dl, pw, tpr);
                for (int sl = wg; sl < P.nslices; sl += nb)
                    update_margin_slice<DT, kNW, GEN>(P, slice_of(sl, P.nslices, nb), cl, h, true,
                                                     h + 1, more, pick2(P.rp, nxt), red, xs, snap_row);
            }
            if (has_gram && more) gram_phase<DT, GEN>(P, pick2(P.G, nxt), h + 1, base, base + nb, lds);
            if (more2) gather_rows<DT>(P, h + 2, gw, ngw);
            if (!grid_barrier_xcd(P.flags, xm, xg, spin)) return;
        } else {
            if (wg == 0) {
                recurrence<ACC, kNT, GEN>(P, pick2(P.G, cur), pick2(P.rp, cur), h, nullptr, nullptr, P.c,
                                     nullptr, dl, pw, tpr);
            } else {
                const int gw1 = gw - kNW, ngw1 = ngw - kNW;
                if (has_gram && more)
                    gram_phase<DT, GEN>(P, pick2(P.G, nxt), h + 1, base + 1, base + nb, lds);
                if (more2) gather_rows<DT>(P, h + 2, gw1, ngw1);
            }
            if (!grid_barrier_xcd(P.flags, xm, xg, spin)) return;
            for (int sl = wg; sl < P.nslices; sl += nb)
                update_margin_slice<DT, kNW, GEN>(P, slice_of(sl, P.nslices, nb), P.c, h, true, h + 1,
                                                 more, pick2(P.rp, nxt), red, xs, snap_row);
            if (!grid_barrier_xcd(P.flags, xm, xg, spin)) return;
        }
        if (snap && wg == 0 && threadIdx.x == 0 && P.t_hist)
            P.t_hist[snap_row + 1] = (int64_t)wall_clock64();
    }
}

// Many problems in one cooperative launch: workgroup w runs problem
// wgmap[w].x as member wgmap[w].y of that problem's group (table[p].gsize
// workgroups, contiguous). Each problem keeps its own workspace and barrier.
// GEN = false when every problem of the batch is plain (logistic, no
// end-to-end rounding), as the single-problem fit compiles that case.
template <int DT, bool GEN>
__global__ __launch_bounds__(kNT) void k_fit_batch(const Dense* table, const int2* wgmap,
                                                   unsigned long long spin) {
    extern __shared__ __align__(16) unsigned char lds[];
    const int2 me = wgmap[blockIdx.x];
    const Dense& P = table[__builtin_amdgcn_readfirstlane(me.x)];
    const int wg = __builtin_amdgcn_readfirstlane(me.y);
    if (P.recur64)
        fit_body<DT, double, true, GEN>(P, wg, P.gsize, spin, lds);
    else
        fit_body<DT, float, true, GEN>(P, wg, P.gsize, spin, lds);
}

// The problem is read in place from the kernel-argument segment (scalar
// loads through the constant cache, as the batched kernel reads its table):
// bound to a reference, the by-value parameter was copied into per-lane
// scratch memory (432 bytes) and every field access became a vector load.
template <int DT, typename ACC, bool GEN>
__global__ __launch_bounds__(kNT) void k_fit(Dense P, unsigned long long spin) {
    extern __shared__ __align__(16) unsigned char lds[];
    (void)P;   // the first kernel argument: at offset 0 of the segment
    const Dense& Pk = *(const Dense*)__builtin_amdgcn_kernarg_segment_ptr();
    fit_body<DT, ACC, true, GEN>(Pk, blockIdx.x, gridDim.x, spin, lds);
}


template <int DT, typename ACC>
inline casgd_status launch_fit_t(const Dense& P, const FitPlan& plan, hipStream_t st) {
    const size_t lds = fit_lds_bytes(P.sb, P.s, (int)sizeof(ACC), slice_width<DT>());
    // the default (logistic, no end-to-end rounding) without run-time mode branches
    auto kern = (P.loss != 0 || P.e2e != 0) ? k_fit<DT, ACC, true> : k_fit<DT, ACC, false>;
    if (lds > 65536) {
        set_error("fused kernel needs %zu bytes of LDS (s*b too large for it)", lds);
        return CASGD_EUNSUPPORTED;
    }
    Dense Pc = P;
    unsigned long long spin = plan.spin;
    void* args[] = {&Pc, &spin};
    CASGD_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(kern), dim3(plan.grid),
                                         dim3(kNT), args, (unsigned)lds, st));
    return CASGD_OK;
}

template <int DT, typename ACC>
inline int fit_max_grid(const Dense& P) {
    const size_t lds = fit_lds_bytes(P.sb, P.s, (int)sizeof(ACC), slice_width<DT>());
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(k_fit<DT, ACC, false>), kNT, lds) != hipSuccess)
        return 0;
    return per_cu * device_cus();
}


template <int DT>
inline const void* batch_kernel_t(bool generic) {
    return generic ? reinterpret_cast<const void*>(k_fit_batch<DT, true>)
                   : reinterpret_cast<const void*>(k_fit_batch<DT, false>);
}

}  // namespace casgd

// Kernels and launchers of the dense s-step SGD path.
//
// Two execution forms share the device functions of dense.hpp,
// recurrence.hpp and fit.hpp:
//  * one launch per phase, stream ordered (kernel boundaries are the
//    synchronisation points): gather of the next block with the margin
//    reduction, Gram, recurrence (multi-workgroup for b = 16, 32, 64, 128),
//    update fused with the next margins;
//  * one persistent cooperative launch for a whole fit (fit.hpp), in three
//    variants (see fit_body), and the batched launch of many problems.
#include <algorithm>
#include <cstring>

#include "internal.hpp"
#include "recurrence.hpp"
#include "fit.hpp"

namespace casgd {

// ------------------------------------------------------------------ kernels

__global__ void k_zero_u32(unsigned* p, int64_t words) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < words) p[i] = 0u;
}

template <int DT>
__global__ __launch_bounds__(kNT) void k_gather(Dense P, uint64_t h, int do_gather,
                                                const float* rp, uint64_t hr, float* r_out) {
    if (do_gather) gather_rows<DT>(P, h, blockIdx.x * kNW + (threadIdx.x >> 6), gridDim.x * kNW);
    if (rp)
        reduce_margins(P, rp, hr, r_out, (int)(blockIdx.x * blockDim.x + threadIdx.x),
                       (int)(gridDim.x * blockDim.x));
}

template <int DT>
__global__ __launch_bounds__(kNT) void k_gram(Dense P, float* Gout, uint64_t h) {
    __shared__ __align__(16) unsigned char lds[kGramLds];
    gram_phase<DT>(P, Gout, h, 0, gridDim.x, lds);
}

// One 128 x 128 LDS tile per workgroup. With a long K range (16 chunks or
// more) the tiles are dealt so that each XCD takes a contiguous run of the
// grouped tile order (workgroup i runs on XCD i % 8): the tiles that run on
// one XCD at the same time then share their row panels in its L2. With a
// short K range the panels are small and the tiles go in row order, which
// measured faster there (consecutive workgroups store neighbouring tiles).
template <int DT>
__global__ __launch_bounds__(kNT) void k_gram128(Dense P, float* Gout, uint64_t h) {
    using T = typename Store<DT>::T;
    __shared__ __align__(16) unsigned char lds[kGram128Lds];
    const int64_t nch = (P.n * (int64_t)sizeof(T) + kChunkB - 1) / kChunkB;
    if (nch < 16) {
        gram_tile128<DT>(P, Gout, h, blockIdx.x, lds);
        return;
    }
    const int Tn = P.t128, id = blockIdx.x, x = id & 7;
    const int L = x * (Tn >> 3) + min(x, Tn & 7) + (id >> 3);
    int TJ, TI;
    grouped_tile128(L, tiles128_per_side(P.sb), TJ, TI);
    gram_tile128_at<DT>(P, Gout, h, TJ, TI, lds);
}

// The 128-tile Gram with K-split tiles, all workgroups resident (a
// cooperative launch of G workgroups, XCD-grouped as above). Tiles 0 .. Tw-1
// of the grouped order are computed whole, G at a time; each of the other
// t128 - Tw tiles is split into S pieces, one per workgroup, after that.
template <int DT>
__global__ __launch_bounds__(kNT) void k_gram128_sk(Dense P, float* Gout, uint64_t h, int Tw,
                                                    int S, unsigned long long spin) {
    __shared__ __align__(16) unsigned char lds[kGram128Lds];
    const unsigned tag = *P.sk_epoch;
    const int G = gridDim.x, id = blockIdx.x, x = id & 7;
    const int v = x * (G >> 3) + min(x, G & 7) + (id >> 3);
    const int NT = tiles128_per_side(P.sb);
    int TJ, TI;
    for (int j = v; j < Tw; j += G) {
        grouped_tile128(j, NT, TJ, TI);
        gram_tile128_at<DT>(P, Gout, h, TJ, TI, lds);
    }
    if (v < (P.t128 - Tw) * S) {
        const int r = v / S, p = v - r * S;
        grouped_tile128(Tw + r, NT, TJ, TI);
        gram_tile128_piece<DT>(P, Gout, h, TJ, TI, p, S,
                               P.sk_slots + (size_t)r * S * kGramSkWords, tag, spin, lds);
    }
}

// Next launch tag of the K-split Gram (never 0, the tag of a cleared word).
// The region is cleared first when its marker word is not set: on first use,
// or when a workspace that held other data (another shape's layout) is
// reused, so a stale word can never carry a future tag. One workgroup.
constexpr unsigned kSkMagic = 0x6b53706cu;

__global__ __launch_bounds__(1024) void k_sk_epoch(unsigned* e, unsigned long long* slots,
                                                   int64_t nwords) {
    __shared__ int fresh;
    if (threadIdx.x == 0) fresh = e[1] != kSkMagic;
    __syncthreads();
    if (fresh) {
        for (int64_t i = threadIdx.x; i < nwords; i += blockDim.x) slots[i] = 0ull;
        if (threadIdx.x == 0) {
            e[0] = 0u;
            e[1] = kSkMagic;
        }
    }
    if (threadIdx.x == 0) {
        const unsigned v = e[0] + 1u;
        e[0] = v ? v : 1u;
    }
}

template <int DT>
__global__ __launch_bounds__(kNT) void k_update(Dense P, const float* c, uint64_t h, int do_update,
                                                uint64_t hn, int do_margin, float* rp_out,
                                                int64_t snap_row) {
    constexpr int KW = slice_width<DT>();
    __shared__ float red[kNW * KW];
    __shared__ float xs[KW];
    update_margin_slice<DT, kNW>(P, blockIdx.x, c, h, do_update != 0, hn, do_margin != 0, rp_out,
                                 red, xs, snap_row);
}

__global__ __launch_bounds__(kNT) void k_margin_reduce(Dense P, const float* rp, uint64_t h,
                                                       float* r_out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= P.sb) return;
    float r = 0.f;
    for (int sl = 0; sl < P.nslices; ++sl) r += rp[(int64_t)sl * P.sb + t];
    r_out[t] = e2e_round(r * pick3(P.sI, slot_of(h))[t], P.e2e);
}

template <typename ACC>
__global__ __launch_bounds__(kNT) void k_recurrence(Dense P, const float* G, const float* rp,
                                                    uint64_t h, const float* r_in,
                                                    const float* y_in, float* c,
                                                    float* delta_out, int tpr) {
    extern __shared__ __align__(16) unsigned char lds[];
    ACC* dl = reinterpret_cast<ACC*>(lds);
    ACC* pw = dl + P.sb;
    recurrence<ACC, kNT>(P, G, rp, h, r_in, y_in, c, delta_out, dl, pw, tpr);
}

// ------------------------------------------------------------------ host

namespace {

template <int DT>
casgd_status launch_gather_t(const Dense& P, uint64_t h, hipStream_t st) {
    const int grid = std::max(1, std::min((P.sb + kNW - 1) / kNW, 4 * device_cus()));
    hipLaunchKernelGGL(k_gather<DT>, dim3(grid), dim3(kNT), 0, st, P, h, 1, nullptr, 0,
                       nullptr);
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

template <int DT>
casgd_status launch_gather_reduce_t(const Dense& P, uint64_t h, int do_gather, const float* rp,
                                    uint64_t hr, float* r_out, hipStream_t st) {
    const int grid = std::max(1, std::min((P.sb + kNW - 1) / kNW, 4 * device_cus()));
    hipLaunchKernelGGL(k_gather<DT>, dim3(grid), dim3(kNT), 0, st, P, h, do_gather, rp, hr, r_out);
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

template <int DT>
casgd_status launch_gram_t(const Dense& P, float* Gout, uint64_t h, hipStream_t st) {
    if (P.gt == 0 || P.s < 2) return CASGD_OK;
    if (P.g128 && P.sk_nslots > 0) {
        // every workgroup resident (the pieces of a tile wait for each other):
        // with more tiles than that, whole rounds first, then the remainder
        // split; pieces keep at least 16 K chunks, at most 16 per tile
        using T = typename Store<DT>::T;
        int per_cu = 0;
        CASGD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_gram128_sk<DT>, kNT, 0));
        const int R = per_cu * device_cus(), Tn = P.t128;
        const int rem = Tn <= R ? Tn : Tn % R;
        const int nch = (int)((P.n * (int64_t)sizeof(T) + kChunkB - 1) / kChunkB);
        const int S = rem > 0 ? std::min({16, nch / 16, R / rem, P.sk_nslots / rem}) : 0;
        if (S >= 2) {
            hipLaunchKernelGGL(k_sk_epoch, dim3(1), dim3(1024), 0, st, P.sk_epoch, P.sk_slots,
                               (int64_t)P.sk_nslots * kGramSkWords);
            CASGD_HIP(hipGetLastError());
            Dense Pc = P;
            int Tw = Tn - rem, Sv = S;
            unsigned long long spin = 1ull << 24;
            const int grid = Tn <= R ? rem * S : R;
            void* args[] = {&Pc, &Gout, &h, &Tw, &Sv, &spin};
            CASGD_HIP(hipLaunchCooperativeKernel((const void*)k_gram128_sk<DT>, dim3(grid),
                                                 dim3(kNT), args, 0, st));
            return CASGD_OK;
        }
    }
    if (P.g128) {
        hipLaunchKernelGGL(k_gram128<DT>, dim3(P.t128), dim3(kNT), 0, st, P, Gout, h);
        CASGD_HIP(hipGetLastError());
        return CASGD_OK;
    }
    const int grid = (P.gna == 4 ? P.gt : 2 * P.gt) * P.ksplit;
    hipLaunchKernelGGL(k_gram<DT>, dim3(grid), dim3(kNT), 0, st, P, Gout, h);
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

template <int DT>
casgd_status launch_update_t(const Dense& P, const float* c, uint64_t h, int do_update,
                             uint64_t hn, int do_margin, float* rp_out, int64_t snap_row,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_update<DT>, dim3(P.nslices), dim3(kNT), 0, st, P, c, h, do_update, hn,
                       do_margin, rp_out, snap_row);
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

template <typename ACC, int NV>
__global__ __launch_bounds__(kNT) void k_rec_multi(Dense P, const float* G, const float* r,
                                                   const float* y, float* c, float* delta_out,
                                                   unsigned long long spin) {
    extern __shared__ __align__(16) unsigned char lds[];
    recurrence_multi<ACC, NV>(P, G, r, y, c, delta_out, P.pub, spin, lds, (int)blockIdx.x);
}

template <typename ACC>
size_t rec_lds(const Dense& P) {
    return (size_t)P.sb * sizeof(ACC) + (size_t)(P.s + 1) * sizeof(ACC);
}

}  // namespace

static const void* batch_kernel(int dtype, bool generic) {
    switch (dtype) {
        case DT_F32: return batch_kernel_f32(generic);
        case DT_BF16: return batch_kernel_bf16(generic);
        case DT_F16: return batch_kernel_f16(generic);
        default: return batch_kernel_fp8(generic);
    }
}

casgd_status run_fit_batch(const Dense* table_dev, const int2* wgmap_dev, int grid, int dtype,
                           size_t lds, unsigned long long spin, bool generic, hipStream_t st) {
    const void* kern = batch_kernel(dtype, generic);
    void* args[] = {const_cast<Dense**>(&table_dev), const_cast<int2**>(&wgmap_dev), &spin};
    CASGD_HIP(hipLaunchCooperativeKernel(kern, dim3(grid), dim3(kNT), args, (unsigned)lds, st));
    return CASGD_OK;
}

int batch_max_grid(int dtype, size_t lds, bool generic) {
    const void* kern = batch_kernel(dtype, generic);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kNT, lds) != hipSuccess) return 0;
    return per_cu * device_cus();
}

size_t fit_lds(const Dense& P, int dtype, int recur64) {
    return fit_lds_bytes(P.sb, P.s, recur64 ? 8 : 4, slice_width_of(dtype));
}

casgd_status run_zero(unsigned* p, int64_t words, hipStream_t st) {
    if (words <= 0) return CASGD_OK;
    const int grid = (int)((words + 255) / 256);
    hipLaunchKernelGGL(k_zero_u32, dim3(grid), dim3(256), 0, st, p, words);
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

casgd_status run_gather(const Dense& P, int dtype, uint64_t h, hipStream_t st) {
    switch (dtype) {
        case DT_F32: return launch_gather_t<DT_F32>(P, h, st);
        case DT_BF16: return launch_gather_t<DT_BF16>(P, h, st);
        case DT_F16: return launch_gather_t<DT_F16>(P, h, st);
        default: return launch_gather_t<DT_FP8>(P, h, st);
    }
}

static casgd_status run_gather_reduce(const Dense& P, int dtype, uint64_t h, int do_gather,
                                      const float* rp, uint64_t hr, float* r_out, hipStream_t st) {
    switch (dtype) {
        case DT_F32: return launch_gather_reduce_t<DT_F32>(P, h, do_gather, rp, hr, r_out, st);
        case DT_BF16: return launch_gather_reduce_t<DT_BF16>(P, h, do_gather, rp, hr, r_out, st);
        case DT_F16: return launch_gather_reduce_t<DT_F16>(P, h, do_gather, rp, hr, r_out, st);
        default: return launch_gather_reduce_t<DT_FP8>(P, h, do_gather, rp, hr, r_out, st);
    }
}

// The multi-workgroup recurrence handles b = 16, 32, 64, 128.
static bool rec_multi_ok(const Dense& P) {
    return P.b == 16 || P.b == 32 || P.b == 64 || P.b == 128;
}

template <typename ACC, int NV>
static casgd_status launch_rec_multi_t(const Dense& P, const float* G, const float* r,
                                       const float* y, float* c, float* delta_out,
                                       unsigned long long spin, hipStream_t st) {
    static_assert(rec_window<NV>() == (NV <= 4 ? 2 : 1), "rec_helpers assumes this window");
    const int R = rec_helpers(P.b, P.s);
    const size_t lds = (size_t)(P.sb + P.s + 1) * sizeof(ACC);
    Dense Pc = P;
    void* args[] = {&Pc, const_cast<float**>(&G), const_cast<float**>(&r), const_cast<float**>(&y),
                    &c, &delta_out, &spin};
    CASGD_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_rec_multi<ACC, NV>),
                                         dim3(1 + R), dim3(kNT), args, (unsigned)lds, st));
    return CASGD_OK;
}

template <typename ACC>
static casgd_status launch_rec_multi_acc(const Dense& P, const float* G, const float* r,
                                         const float* y, float* c, float* delta_out,
                                         unsigned long long spin, hipStream_t st) {
    switch (P.b) {
        case 16: return launch_rec_multi_t<ACC, 1>(P, G, r, y, c, delta_out, spin, st);
        case 32: return launch_rec_multi_t<ACC, 2>(P, G, r, y, c, delta_out, spin, st);
        case 64: return launch_rec_multi_t<ACC, 4>(P, G, r, y, c, delta_out, spin, st);
        default: return launch_rec_multi_t<ACC, 8>(P, G, r, y, c, delta_out, spin, st);
    }
}

casgd_status run_recurrence_multi(const Dense& P, const float* G, const float* r, const float* y,
                                  float* c, float* delta_out, bool fp64, unsigned long long spin,
                                  hipStream_t st) {
    return fp64 ? launch_rec_multi_acc<double>(P, G, r, y, c, delta_out, spin, st)
                : launch_rec_multi_acc<float>(P, G, r, y, c, delta_out, spin, st);
}

casgd_status run_gram(const Dense& P, int dtype, float* Gout, uint64_t h, hipStream_t st) {
    switch (dtype) {
        case DT_F32: return launch_gram_t<DT_F32>(P, Gout, h, st);
        case DT_BF16: return launch_gram_t<DT_BF16>(P, Gout, h, st);
        case DT_F16: return launch_gram_t<DT_F16>(P, Gout, h, st);
        default: return launch_gram_t<DT_FP8>(P, Gout, h, st);
    }
}

static casgd_status run_update_margin(const Dense& P, int dtype, const float* c, uint64_t h,
                                      int do_update, uint64_t hn, int do_margin, float* rp_out,
                                      int64_t snap_row, hipStream_t st) {
    switch (dtype) {
        case DT_F32:
            return launch_update_t<DT_F32>(P, c, h, do_update, hn, do_margin, rp_out, snap_row, st);
        case DT_BF16:
            return launch_update_t<DT_BF16>(P, c, h, do_update, hn, do_margin, rp_out, snap_row, st);
        case DT_F16:
            return launch_update_t<DT_F16>(P, c, h, do_update, hn, do_margin, rp_out, snap_row, st);
        default:
            return launch_update_t<DT_FP8>(P, c, h, do_update, hn, do_margin, rp_out, snap_row, st);
    }
}

casgd_status run_margin(const Dense& P, int dtype, uint64_t h, float* rp_out, hipStream_t st) {
    return run_update_margin(P, dtype, nullptr, 0, 0, h, 1, rp_out, -1, st);
}

casgd_status run_update(const Dense& P, int dtype, const float* c, uint64_t h, hipStream_t st) {
    return run_update_margin(P, dtype, c, h, 1, 0, 0, nullptr, -1, st);
}

casgd_status run_margin_reduce(const Dense& P, const float* rp, uint64_t h, float* r_out,
                               hipStream_t st) {
    const int grid = (P.sb + kNT - 1) / kNT;
    hipLaunchKernelGGL(k_margin_reduce, dim3(grid), dim3(kNT), 0, st, P, rp, h, r_out);
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

casgd_status run_recurrence(const Dense& P, const float* G, const float* rp, uint64_t h,
                            const float* r_in, const float* y_in, float* c, float* delta_out,
                            bool fp64, hipStream_t st) {
    const int tpr = recurrence_tpr(kNT, P.b);
    if (fp64) {
        const size_t lds = rec_lds<double>(P);
        if (lds > 65536) {
            set_error("recurrence needs %zu bytes of LDS", lds);
            return CASGD_EUNSUPPORTED;
        }
        hipLaunchKernelGGL(k_recurrence<double>, dim3(1), dim3(kNT), lds, st, P, G, rp, h, r_in,
                           y_in, c, delta_out, tpr);
    } else {
        const size_t lds = rec_lds<float>(P);
        hipLaunchKernelGGL(k_recurrence<float>, dim3(1), dim3(kNT), lds, st, P, G, rp, h, r_in,
                           y_in, c, delta_out, tpr);
    }
    CASGD_HIP(hipGetLastError());
    return CASGD_OK;
}

static int fit_max_grid_dt(const Dense& P, int dtype, int recur64) {
    switch (dtype) {
        case DT_F32: return fit_max_grid_f32(P, recur64);
        case DT_BF16: return fit_max_grid_bf16(P, recur64);
        case DT_F16: return fit_max_grid_f16(P, recur64);
        default: return fit_max_grid_fp8(P, recur64);
    }
}

bool choose_gram128(const Dense& P, int dtype, int gram_tile, int gram_workgroups) {
    if (P.s < 2) return false;
    if (gram_tile == 128) return true;
    if (gram_tile == 64) return false;
    DenseLayout L;
    dense_layout(P.n, dtype, P.b, P.s, &L);
    // measured on MI355X: with low-precision storage the LDS tiles win from
    // about one tile per two Gram workgroups on; FP32 (four MFMAs per
    // 16-byte operand) needs one per workgroup
    return dtype == CASGD_F32 ? L.n128 >= gram_workgroups : 2 * L.n128 >= gram_workgroups;
}

casgd_status plan_fit(const Dense& P, int dtype, const casgd_opts* o, int64_t H, FitPlan* plan) {
    const int64_t sb = P.sb;
    int prec = o ? o->recur_prec : 0;
    if (prec != 0 && prec != 32 && prec != 64) {
        set_error("recur_prec must be 0, 32 or 64 (got %d)", prec);
        return CASGD_EINVAL;
    }
    plan->recur64 = P.e2e == 0 && (prec == 64 || (prec == 0 && sb >= 512));
    plan->exec_mode = (o && o->exec_mode) ? o->exec_mode : 1;
    if (plan->exec_mode != 1 && plan->exec_mode != 2) {
        set_error("exec_mode must be 0, 1 or 2 (got %d)", plan->exec_mode);
        return CASGD_EINVAL;
    }
    plan->spin = (o && o->spin_limit > 0) ? (unsigned long long)o->spin_limit : (1ull << 24);
    // Strict block-lower Gram bytes read by each recurrence.
    const double gl_bytes = 4.0 * P.b * (double)P.b * P.s * (P.s - 1) / 2.0;
    // Automatic variant (measured on MI355X over b = 16 .. 128, s = 2 .. 32):
    // the multi-workgroup recurrence from s = 4 on, one recurrence workgroup
    // beside the Gram builders at s = 2 and 3, and every workgroup running
    // the recurrence itself only for other b with a small G_L (or s = 1).
    const bool multi_ok = rec_multi_ok(P) && P.s > 1;
    int variant = (o && o->fused_variant)
                      ? o->fused_variant
                      : (multi_ok ? (P.s >= 4 ? 3 : 2) : (gl_bytes <= 256.0 * 1024 ? 1 : 2));
    if (variant < 1 || variant > 3) {
        set_error("fused_variant must be 0, 1, 2 or 3 (got %d)", variant);
        return CASGD_EINVAL;
    }
    if (variant == 3 && !multi_ok) {
        set_error("fused_variant 3 needs b = 16, 32, 64 or 128 and s > 1");
        return CASGD_EUNSUPPORTED;
    }
    plan->variant = variant;
    plan->grid = 0;
    const int gram_tile = o ? o->gram_tile : 0;
    if (gram_tile != 0 && gram_tile != 64 && gram_tile != 128) {
        set_error("gram_tile must be 0, 64 or 128 (got %d)", gram_tile);
        return CASGD_EINVAL;
    }
    plan->gram128 = choose_gram128(P, dtype, gram_tile, device_cus());
    if (plan->exec_mode == 2) return CASGD_OK;
    const size_t lds = fit_lds_bytes(P.sb, P.s, plan->recur64 ? 8 : 4, slice_width_of(dtype));
    if (lds > 65536) {
        plan->exec_mode = 2;  // the fused kernel cannot hold this recurrence in LDS
        return CASGD_OK;
    }
    const int maxg = fit_max_grid_dt(P, dtype, plan->recur64);
    if (maxg <= 0) {
        plan->exec_mode = 2;
        return CASGD_OK;
    }
    DenseLayout L128;
    dense_layout(P.n, dtype, P.b, P.s, &L128);
    const int units = P.s > 1 ? (plan->gram128 ? L128.n128 : (P.gna == 4 ? P.gt : 2 * P.gt) * P.ksplit)
                              : 0;
    // workgroups that run the recurrence while the others build the next Gram
    const int nrec = variant == 3 ? 1 + rec_helpers(P.b, P.s) : (variant == 2 ? 1 : 0);
    int want = std::max(P.nslices, units + nrec);
    want = std::max(want, nrec + 1);
    if (o && o->grid_blocks > 0) want = o->grid_blocks;
    plan->grid = std::min(want, maxg);
    if (plan->grid < nrec + 1) plan->exec_mode = 2;
    (void)H;
    return CASGD_OK;
}

casgd_status run_fit(const Dense& P0, int dtype, uint64_t h0, int64_t H, const FitPlan& plan,
                     hipStream_t st) {
    if (H <= 0) return CASGD_OK;
    Dense P = P0;
    P.g128 = plan.gram128;
    casgd_status rc;
    // Split-K counters must start at zero (they reset themselves after use,
    // but a launch that stopped early may leave them set).
    if ((rc = run_zero(P.tile_cnt, 2 * P.ntiles, st)) != CASGD_OK) return rc;
    if (plan.exec_mode == 1) {
        // Barrier words start from zero for every fused launch.
        if ((rc = run_zero(P.flags + FLAG_BAR_COUNT, FLAG_WORDS - FLAG_BAR_COUNT, st)) != CASGD_OK)
            return rc;
        if (plan.variant == 3 &&
            (rc = run_zero(reinterpret_cast<unsigned*>(P.pub), (int64_t)P.sb * 8, st)) != CASGD_OK)
            return rc;
        Dense Q = P;
        Q.h0 = h0;
        Q.H = H;
        Q.variant = plan.variant;
        Q.gsize = plan.grid;
        Q.recur64 = plan.recur64;
        Q.g128 = plan.gram128;
        Q.tpr = recurrence_tpr(kNT, P.b);
        switch (dtype) {
            case DT_F32: return launch_fit_f32(Q, plan, st);
            case DT_BF16: return launch_fit_bf16(Q, plan, st);
            case DT_F16: return launch_fit_f16(Q, plan, st);
            default: return launch_fit_fp8(Q, plan, st);
        }
    }
    // Stream-ordered: gather(h0), margin(h0); then per outer: gram(h),
    // gather(h+1) (with the reduction of the margins of h when the
    // multi-workgroup recurrence runs), recurrence(h), update(h) fused with
    // margin(h+1).
    const bool multi = rec_multi_ok(P);
    if ((rc = run_gather(P, dtype, h0, st)) != CASGD_OK) return rc;
    if ((rc = run_update_margin(P, dtype, nullptr, 0, 0, h0, 1, P.rp[0], -1, st)) != CASGD_OK)
        return rc;
    // the recurrence's exchange words start from zero (each launch clears them)
    if (multi && (rc = run_zero(reinterpret_cast<unsigned*>(P.pub), (int64_t)P.sb * 8, st)) != CASGD_OK)
        return rc;
    for (int64_t hh = 0; hh < H; ++hh) {
        const uint64_t h = h0 + (uint64_t)hh;
        const bool more = hh + 1 < H;
        const bool snap = P.snap_every > 0 && ((hh + 1) % P.snap_every) == 0;
        const int64_t snap_row = snap ? (hh + 1) / P.snap_every - 1 : -1;
        if ((rc = run_gram(P, dtype, P.G[0], h, st)) != CASGD_OK) return rc;
        if (multi) {
            if ((rc = run_gather_reduce(P, dtype, h + 1, more ? 1 : 0, P.rp[0], h, P.r, st)) !=
                CASGD_OK)
                return rc;
            if ((rc = run_recurrence_multi(P, P.G[0], P.r, P.yI[slot_of_host(h)], P.c, nullptr,
                                    plan.recur64 != 0, plan.spin, st)) != CASGD_OK)
                return rc;
        } else {
            if (more && (rc = run_gather(P, dtype, h + 1, st)) != CASGD_OK) return rc;
            if ((rc = run_recurrence(P, P.G[0], P.rp[0], h, nullptr, nullptr, P.c, nullptr,
                                     plan.recur64 != 0, st)) != CASGD_OK)
                return rc;
        }
        if ((rc = run_update_margin(P, dtype, P.c, h, 1, h + 1, more ? 1 : 0, P.rp[0], snap_row,
                                    st)) != CASGD_OK)
            return rc;
    }
    return CASGD_OK;
}

}  // namespace casgd

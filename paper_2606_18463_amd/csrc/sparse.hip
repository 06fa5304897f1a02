// Sparse (CSR) s-step SGD with lambda lanes: fused persistent kernel and host
// side (workspace layout, head/tail preparation, dispatch).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.hpp"
#include "misc.hpp"
#include "sparse.hpp"

namespace casgd {

// ------------------------------------------------------------------ kernels

__global__ void k_colcount(const int32_t* ci, int64_t nnz, unsigned* cnt) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz;
         p += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(cnt + ci[p], 1u);
}

struct LaneParams {
    double beta[kMaxLanes];
    float beta_s[kMaxLanes];
};

__global__ void k_set_lanes(LaneParams p, int L, double* lbeta, float* lbs) {
    const int l = threadIdx.x;
    if (l < L) {
        lbeta[l] = p.beta[l];
        lbs[l] = p.beta_s[l];
    }
}

// LDS: lane deltas and decay powers of the recurrence, then the per-wave
// head-row buffers of the gather, which the recurrence workgroups use for
// their reduction buffer instead (phases never overlap in a workgroup).
__host__ __device__ inline size_t sparse_lds_bytes(int sb, int s, int acc_bytes, int Hp) {
    size_t off = (size_t)sb * kLanesPerRecWG * acc_bytes;
    off += (size_t)kLanesPerRecWG * (s + 1) * acc_bytes;
    off = (off + 15) & ~(size_t)15;
    const size_t rows = (size_t)kNW * Hp * 4;
    const size_t red = (size_t)kRecRows * kLanesPerRecWG * (kNT / 4) * acc_bytes;
    off += rows > red ? rows : red;
    // the head-panel Gram phase reuses the same memory
    return off < kGramLds ? kGramLds : off;
}

// Per outer iteration h, with R recurrence workgroups (K per group of
// kLanesPerRecWG lanes, splitting the rows of each block) and the remaining
// workgroups as workers:
//   P1  recurrence(h)            | Gram head(h+1), gather(h+2), buckets(h+1)
//   --  barrier
//   P2  update(h), Gram tail(h+1)
//   --  barrier
//   P3  margins(h+1), clear buckets(h)
//   --  barrier
template <typename ACC>
__global__ __launch_bounds__(kNT) void k_sparse_fit(Sparse S_arg, uint64_t h0, int64_t H,
                                                    unsigned long long spin, int K, int R) {
    extern __shared__ __align__(16) unsigned char lds[];
    // The problem is read in place from the kernel-argument segment (scalar
    // loads through the constant cache): bound to references, the by-value
    // parameter was copied into per-lane scratch memory (856 bytes).
    (void)S_arg;   // the first kernel argument: at offset 0 of the segment
    const Sparse& S = *(const Sparse*)__builtin_amdgcn_kernarg_segment_ptr();
    constexpr int NL = kLanesPerRecWG;
    ACC* dl = reinterpret_cast<ACC*>(lds);
    ACC* pw = dl + (size_t)S.sb * NL;
    size_t off = (size_t)S.sb * NL * sizeof(ACC) + (size_t)NL * (S.s + 1) * sizeof(ACC);
    off = (off + 15) & ~(size_t)15;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float* hrow = reinterpret_cast<float*>(lds + off) + (size_t)wave * S.Hp;
    ACC* red = reinterpret_cast<ACC*>(lds + off);
    // outside the recurrence the lane deltas' space holds one row of G per wave
    float* rowbuf = reinterpret_cast<float*>(lds) + (size_t)wave * S.sb;

    const int nb = gridDim.x, wg = blockIdx.x;
    const int gw = wg * kNW + wave, ngw = nb * kNW;
    const int gtid = wg * kNT + threadIdx.x, nthr = nb * kNT;

    if (threadIdx.x == 0 && wg == 0 && S.t_hist) S.t_hist[0] = (int64_t)wall_clock64();
    // Prologue: rows of h0 and h0+1; buckets and Gram of h0; margins of h0.
    // The first barrier also completes the XCD census; every later one
    // writes each XCD's L2 back once (grid_barrier_xcd).
    xcd_census_add(S.flags, false);
    sparse_gather(S, h0, gw, ngw, hrow);
    if (H > 1) sparse_gather(S, h0 + 1, gw, ngw, hrow);
    if (!grid_barrier(S.flags, wg, nb, spin)) return;
    unsigned xm, xg, xs_unused;
    xcd_census_read(S.flags, xm, xg, xs_unused);
    sparse_bucket(S, h0, gtid, nthr);
    gram_phase<DT_F32>(S.gram, spick2(S.G, (int)(h0 & 1)), h0, 0, nb, lds);
    if (!grid_barrier_xcd(S.flags, xm, xg, spin)) return;
    sparse_gram_tail(S, h0, spick2(S.G, (int)(h0 & 1)), gw, ngw, rowbuf);
    sparse_margins(S, h0, reinterpret_cast<float*>(lds));
    if (!grid_barrier_xcd(S.flags, xm, xg, spin)) return;

    for (int64_t hh = 0; hh < H; ++hh) {
        const uint64_t h = h0 + (uint64_t)hh;
        const bool more = hh + 1 < H, more2 = hh + 2 < H;
        const bool snap = S.snap_every > 0 && ((hh + 1) % S.snap_every) == 0;
        const int64_t snap_row = snap ? (hh + 1) / S.snap_every - 1 : -1;
        auto mark = [&](int k) {
            if (S.ptrace && threadIdx.x == 0 && hh < S.ptrace_outer)
                S.ptrace[hh * 8 + k] = (int64_t)wall_clock64();
        };
        if (wg == 0) mark(0);
        if (wg < R) {
            const int l0 = (wg / K) * NL;
            sparse_recurrence<ACC, kNT>(S, spick2(S.G, (int)(h & 1)), h, l0, min(NL, S.L - l0),
                                        wg % K, K, dl, pw, red, spin);
            if (wg == 0) mark(1);
        } else {
            const int w0 = (wg - R) * kNW + wave, nw = (nb - R) * kNW;
            const int t0 = (wg - R) * kNT + threadIdx.x, nt = (nb - R) * kNT;
            if (more) {
                gram_phase<DT_F32>(S.gram, spick2(S.G, (int)((h + 1) & 1)), h + 1, R, nb, lds);
                sparse_bucket(S, h + 1, t0, nt);
            }
            if (more2) sparse_gather(S, h + 2, w0, nw, hrow);
            if (wg == R) mark(2);
        }
        if (!grid_barrier_xcd(S.flags, xm, xg, spin)) return;
        if (wg == 0) mark(3);
        if (wg < R) sparse_pub_clear(S, (wg / K) * NL, min(NL, S.L - (wg / K) * NL), wg % K, K);
        // the wave's scratch for the tail update: its head-row buffer
        sparse_update(S, h, gw, ngw, gtid, nthr, snap_row, reinterpret_cast<int2*>(hrow),
                      reinterpret_cast<float*>(lds));
        if (wg == 0) mark(4);
        if (more) sparse_gram_tail(S, h + 1, spick2(S.G, (int)((h + 1) & 1)), gw, ngw, rowbuf);
        if (wg == 0) mark(5);
        if (!grid_barrier_xcd(S.flags, xm, xg, spin)) return;
        if (wg == 0) mark(6);
        if (more) sparse_margins(S, h + 1, reinterpret_cast<float*>(lds));
        sparse_clear_buckets(S, h, gtid, nthr);
        if (!grid_barrier_xcd(S.flags, xm, xg, spin)) return;
        if (wg == 0) mark(7);
        if (snap && wg == 0 && threadIdx.x == 0 && S.t_hist)
            S.t_hist[snap_row + 1] = (int64_t)wall_clock64();
    }
}

// ------------------------------------------------------------------ host

namespace {

struct SparseLayout {
    int sb, sbpad, maxlen, L;
    DenseLayout gl;  // Gram tiles over the head panel (n = kHeadMax, FP32)
    size_t off_flags, off_prep, off_tilecnt, off_G0, off_G1, off_Gpart, off_r, off_c, off_pub, off_lbeta, off_lbs,
        off_headid, off_headcol, off_colcnt, off_Yh[3], off_tcol[3], off_tval[3], off_tlen[3],
        off_yI[3], off_bcnt[2], off_bent[2], off_tlist[2], off_tlcnt, total;
};

size_t a256(size_t v) { return (v + 255) & ~(size_t)255; }

void sparse_layout(int64_t n, int b, int s, int L, int maxlen, SparseLayout* S) {
    S->sb = b * s;
    S->maxlen = std::max(1, maxlen);
    S->L = L;
    dense_layout(kHeadMax, CASGD_F32, b, s, &S->gl);
    S->sbpad = S->gl.ts * kTile;
    const size_t sb = S->sb;
    size_t off = 0;
    auto take = [&](size_t& o, size_t bytes) { o = off; off = a256(off + bytes); };
    take(S->off_flags, FLAG_WORDS * 4);
    take(S->off_prep, 256);   // the Prepared record (fixed offset: flags come first)
    take(S->off_tilecnt, (size_t)S->gl.ntiles * 2 * 4);
    take(S->off_G0, sb * sb * 4);
    take(S->off_G1, sb * sb * 4);
    take(S->off_Gpart, S->gl.ksplit > 1 ? (size_t)S->gl.ntiles * S->gl.ksplit * 4096 * 4 : 0);
    take(S->off_r, sb * L * 4);
    take(S->off_c, sb * L * 4);
    take(S->off_pub, sb * L * 16);
    take(S->off_lbeta, (size_t)kMaxLanes * 8);
    take(S->off_lbs, (size_t)kMaxLanes * 4);
    take(S->off_headid, (size_t)n * 4);
    take(S->off_headcol, (size_t)kHeadMax * 4);
    take(S->off_colcnt, (size_t)n * 4);
    for (int k = 0; k < 3; ++k) {
        take(S->off_Yh[k], (size_t)S->sbpad * kHeadMax * 4);
        take(S->off_tcol[k], sb * S->maxlen * 4);
        take(S->off_tval[k], sb * S->maxlen * 4);
        take(S->off_tlen[k], sb * 4);
        take(S->off_yI[k], sb * 4);
    }
    for (int k = 0; k < 2; ++k) {
        take(S->off_bcnt[k], (size_t)n * 4);
        take(S->off_bent[k], (size_t)n * kBucketCap * 8);
        take(S->off_tlist[k], (size_t)n * 4);
    }
    take(S->off_tlcnt, 2 * 4);
    S->total = off;
}

// What casgd_sparse_prepare decided for a workspace (X, b, s, lanes, the
// head split), stored in the workspace itself right after the flag words:
// the library keeps no host state between calls.
struct Prepared {
    uint64_t magic;
    const void* rp;
    const void* ci;
    const void* va;
    int64_t m, n, nnz;
    int b, s, L, H, Hp, maxlen;
};
constexpr uint64_t kPrepMagic = 0x63617367645f7370ull;   // "casgd_sp"
constexpr size_t kPrepOffset = (FLAG_WORDS * 4 + 255) & ~(size_t)255;
static_assert(sizeof(Prepared) <= 256, "the prepared record has 256 bytes");

casgd_status csr_maxlen(const casgd_matrix* X, int* maxlen) {
    std::vector<int64_t> rp((size_t)X->m + 1);
    CASGD_HIP(hipMemcpy(rp.data(), X->row_ptr, rp.size() * 8, hipMemcpyDeviceToHost));
    int64_t mx = 0;
    for (int64_t i = 0; i < X->m; ++i) mx = std::max(mx, rp[i + 1] - rp[i]);
    if (rp[0] != 0 || rp[X->m] != X->nnz) {
        set_error("row_ptr must start at 0 and end at nnz");
        return CASGD_EINVAL;
    }
    if (mx > (1 << 20)) {
        set_error("CSR rows longer than 2^20 entries are not supported");
        return CASGD_EUNSUPPORTED;
    }
    *maxlen = (int)mx;
    return CASGD_OK;
}

casgd_status check_sparse_args(const casgd_matrix* X, int32_t b, int32_t s, int32_t L) {
    if (!X || X->layout != CASGD_CSR || !X->row_ptr || X->m < 1 || X->n < 1 ||
        (X->nnz > 0 && (!X->col_idx || !X->values))) {
        set_error("expected a CSR matrix");
        return CASGD_EINVAL;
    }
    if (X->dtype != CASGD_F32) {
        set_error("CSR values must be FP32");
        return CASGD_EUNSUPPORTED;
    }
    if (b < 1 || s < 1 || L < 1) {
        set_error("b, s and the lane count must be >= 1");
        return CASGD_EINVAL;
    }
    if ((int64_t)b * s > 4096 || L > kMaxLanes) {
        set_error("s*b <= 4096 and at most %d lanes are supported", kMaxLanes);
        return CASGD_EUNSUPPORTED;
    }
    if (b % 4) {
        set_error("the CSR path needs b to be a multiple of 4");
        return CASGD_EUNSUPPORTED;
    }
    return CASGD_OK;
}

template <typename T>
T* at(void* ws, size_t off) {
    return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

}  // namespace

casgd_status sparse_workspace_size(const casgd_matrix* X, int32_t b, int32_t s, int32_t lanes,
                                   size_t* bytes) {
    casgd_status rc;
    if ((rc = check_sparse_args(X, b, s, lanes)) != CASGD_OK) return rc;
    int maxlen = 0;
    if ((rc = csr_maxlen(X, &maxlen)) != CASGD_OK) return rc;
    SparseLayout L;
    sparse_layout(X->n, b, s, lanes, maxlen, &L);
    *bytes = L.total;
    return CASGD_OK;
}

casgd_status sparse_prepare(const casgd_matrix* X, int32_t b, int32_t s, int32_t lanes, void* ws,
                            size_t ws_bytes, void* stream) {
    casgd_status rc;
    if ((rc = check_sparse_args(X, b, s, lanes)) != CASGD_OK) return rc;
    int maxlen = 0;
    if ((rc = csr_maxlen(X, &maxlen)) != CASGD_OK) return rc;
    SparseLayout SL;
    sparse_layout(X->n, b, s, lanes, maxlen, &SL);
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) || ws_bytes < SL.total) {
        set_error("workspace missing, misaligned or too small (%zu bytes needed)", SL.total);
        return ws_bytes < SL.total ? CASGD_ENOMEM : CASGD_EINVAL;
    }
    hipStream_t st = (hipStream_t)stream;
    unsigned* cnt = at<unsigned>(ws, SL.off_colcnt);
    CASGD_HIP(hipMemsetAsync(cnt, 0, (size_t)X->n * 4, st));
    if (X->nnz > 0) {
        const int grid = (int)std::min<int64_t>((X->nnz + 255) / 256, 4096);
        hipLaunchKernelGGL(k_colcount, dim3(grid), dim3(256), 0, st, X->col_idx, X->nnz, cnt);
        CASGD_HIP(hipGetLastError());
    }
    std::vector<unsigned> hc((size_t)X->n);
    CASGD_HIP(hipMemcpyAsync(hc.data(), cnt, hc.size() * 4, hipMemcpyDeviceToHost, st));
    CASGD_HIP(hipStreamSynchronize(st));
    // Head: the most frequent columns whose expected occurrence in one block
    // of s*b sampled rows is at least one, at least 128 (or n) and at most
    // kHeadMax of them.
    std::vector<int32_t> order((size_t)X->n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t c) { return hc[a] > hc[c]; });
    const double sb = (double)b * s;
    int H = 0;
    while (H < (int)X->n && H < kHeadMax && (double)hc[order[H]] * sb / (double)X->m >= 1.0) ++H;
    H = std::max(H, (int)std::min<int64_t>(X->n, 128));
    H = std::min(H, kHeadMax);
    std::vector<int32_t> head_id((size_t)X->n, -1);
    std::vector<int32_t> head_col(kHeadMax, 0);
    std::vector<int32_t> sel(order.begin(), order.begin() + H);
    std::sort(sel.begin(), sel.end());
    for (int i = 0; i < H; ++i) {
        head_id[sel[i]] = i;
        head_col[i] = sel[i];
    }
    CASGD_HIP(hipMemcpyAsync(at<int32_t>(ws, SL.off_headid), head_id.data(), head_id.size() * 4,
                             hipMemcpyHostToDevice, st));
    CASGD_HIP(hipMemcpyAsync(at<int32_t>(ws, SL.off_headcol), head_col.data(),
                             head_col.size() * 4, hipMemcpyHostToDevice, st));
    for (int k = 0; k < 2; ++k)
        CASGD_HIP(hipMemsetAsync(at<unsigned>(ws, SL.off_bcnt[k]), 0, (size_t)X->n * 4, st));
    CASGD_HIP(hipMemsetAsync(ws, 0, FLAG_WORDS * 4, st));
    const Prepared P{kPrepMagic, X->row_ptr, X->col_idx, X->values, X->m, X->n, X->nnz, b, s,
                     lanes, H, (H + 127) / 128 * 128, maxlen};
    CASGD_HIP(hipMemcpyAsync(at<char>(ws, SL.off_prep), &P, sizeof P, hipMemcpyHostToDevice, st));
    CASGD_HIP(hipStreamSynchronize(st));
    return CASGD_OK;
}

casgd_status sparse_fit(const casgd_matrix* X, const float* y, float* x_lanes,
                        const double* lambdas_host, int32_t L, double eta, int32_t b, int32_t s,
                        uint64_t seed, uint64_t outer_begin, int64_t n_outer,
                        const casgd_opts* opts, void* ws, size_t ws_bytes, void* stream) {
    casgd_status rc;
    if ((rc = check_sparse_args(X, b, s, L)) != CASGD_OK) return rc;
    if (!y || !x_lanes || !lambdas_host) {
        set_error("y, x and lambdas must not be NULL");
        return CASGD_EINVAL;
    }
    if (!(eta > 0) || !std::isfinite(eta) || n_outer < 0) {
        set_error("need eta > 0 and n_outer >= 0");
        return CASGD_EINVAL;
    }
    for (int l = 0; l < L; ++l)
        if (!(lambdas_host[l] >= 0) || !std::isfinite(lambdas_host[l])) {
            set_error("lambda[%d] must be finite and >= 0", l);
            return CASGD_EINVAL;
        }
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255) || ws_bytes < kPrepOffset + 256) {
        set_error("workspace missing, misaligned or too small");
        return CASGD_EINVAL;
    }
    // the record casgd_sparse_prepare left in the workspace (written once,
    // before that call returned; a small synchronous read)
    Prepared P;
    CASGD_HIP(hipMemcpy(&P, at<char>(ws, kPrepOffset), sizeof P, hipMemcpyDeviceToHost));
    if (P.magic != kPrepMagic) {
        set_error("workspace not prepared: call casgd_sparse_prepare for this X, b, s first");
        return CASGD_EINVAL;
    }
    if (P.rp != X->row_ptr || P.ci != X->col_idx || P.va != X->values || P.m != X->m ||
        P.n != X->n || P.b != b || P.s != s || L > P.L) {
        set_error("workspace was prepared for a different X, b, s or fewer lanes");
        return CASGD_EINVAL;
    }
    SparseLayout SL;
    sparse_layout(X->n, b, s, P.L, P.maxlen, &SL);
    if (ws_bytes < SL.total) {
        set_error("workspace too small");
        return CASGD_ENOMEM;
    }
    if (n_outer == 0) return CASGD_OK;
    hipStream_t st = (hipStream_t)stream;

    Sparse S;
    std::memset(&S, 0, sizeof S);
    S.rp = X->row_ptr;
    S.ci = X->col_idx;
    S.va = static_cast<const float*>(X->values);
    S.y = y;
    S.x = x_lanes;
    S.m = X->m;
    S.n = X->n;
    S.L = L;
    S.b = b;
    S.s = s;
    S.sb = b * s;
    S.seed = seed;
    S.alpha_d = eta / b;
    S.lbeta = at<double>(ws, SL.off_lbeta);
    S.lbs = at<float>(ws, SL.off_lbs);
    S.head_id = at<int32_t>(ws, SL.off_headid);
    S.head_col = at<int32_t>(ws, SL.off_headcol);
    S.H = P.H;
    S.Hp = P.Hp;
    S.maxlen = SL.maxlen;
    S.flags = at<unsigned>(ws, SL.off_flags);
    S.loss = opts ? opts->loss : 0;
    if ((rc = check_loss(S.loss)) != CASGD_OK) return rc;
    if (opts && opts->e2e) {
        set_error("the end-to-end low-precision emulation needs a dense X");
        return CASGD_EUNSUPPORTED;
    }
    for (int k = 0; k < 3; ++k) {
        S.Yh[k] = at<float>(ws, SL.off_Yh[k]);
        S.tcol[k] = at<int32_t>(ws, SL.off_tcol[k]);
        S.tval[k] = at<float>(ws, SL.off_tval[k]);
        S.tlen[k] = at<int32_t>(ws, SL.off_tlen[k]);
        S.yI[k] = at<float>(ws, SL.off_yI[k]);
    }
    for (int k = 0; k < 2; ++k) {
        S.bcnt[k] = at<unsigned>(ws, SL.off_bcnt[k]);
        S.bent[k] = at<int2>(ws, SL.off_bent[k]);
        S.tlist[k] = at<int32_t>(ws, SL.off_tlist[k]);
    }
    S.G[0] = at<float>(ws, SL.off_G0);
    S.G[1] = at<float>(ws, SL.off_G1);
    S.r = at<float>(ws, SL.off_r);
    S.c = at<float>(ws, SL.off_c);
    S.pub = at<unsigned long long>(ws, SL.off_pub);
    S.tlcnt = at<unsigned>(ws, SL.off_tlcnt);
    if (opts && opts->snapshot_every > 0) {
        if (!opts->x_history) {
            set_error("snapshot_every > 0 needs x_history");
            return CASGD_EINVAL;
        }
        S.snap_every = opts->snapshot_every;
        S.x_hist = opts->x_history;
        S.t_hist = opts->t_history;
    }
    if (opts && opts->phase_trace && opts->phase_trace_outer > 0) {
        S.ptrace = opts->phase_trace;
        S.ptrace_outer = opts->phase_trace_outer;
    }
    // Gram view over the head panel.
    Dense& Gv = S.gram;
    Gv.b = b;
    Gv.s = s;
    Gv.sb = S.sb;
    Gv.ldg = S.sb;
    Gv.n = P.H;
    Gv.ldy = P.Hp;
    Gv.m = X->m;
    Gv.ts = SL.gl.ts;
    Gv.ntiles = SL.gl.ntiles;
    Gv.gt = SL.gl.gt;
    Gv.bt = SL.gl.bt;
    Gv.gna = SL.gl.gna;
    {
        // K = H is short: split it only up to the partial buffer's capacity,
        // keeping at least 64 K elements per split
        const int64_t kpad = (P.H + 15) / 16 * 16;
        const int ks = std::max(1, std::min(SL.gl.ksplit, (int)(kpad / 64)));
        Gv.kchunk = ((kpad + ks - 1) / ks + 15) / 16 * 16;
        Gv.ksplit = (int)((kpad + Gv.kchunk - 1) / Gv.kchunk);
    }
    Gv.flags = S.flags;
    Gv.tile_cnt = at<unsigned>(ws, SL.off_tilecnt);
    Gv.Gpart = at<float>(ws, SL.off_Gpart);
    for (int k = 0; k < 3; ++k) {
        Gv.Y[k] = S.Yh[k];
        Gv.sI[k] = S.yI[k];  // never read: no row scales
        Gv.yI[k] = S.yI[k];
    }

    // Lane constants.
    LaneParams lp;
    std::memset(&lp, 0, sizeof lp);
    for (int l = 0; l < L; ++l) {
        lp.beta[l] = 1.0 - eta * lambdas_host[l];
        lp.beta_s[l] = (float)std::pow(lp.beta[l], (double)s);
    }
    hipLaunchKernelGGL(k_set_lanes, dim3(1), dim3(kMaxLanes), 0, st, lp, L,
                       const_cast<double*>(S.lbeta), const_cast<float*>(S.lbs));
    CASGD_HIP(hipGetLastError());
    if ((rc = run_zero(Gv.tile_cnt, 2 * Gv.ntiles, st)) != CASGD_OK) return rc;
    if ((rc = run_zero(S.tlcnt, 2, st)) != CASGD_OK) return rc;
    if ((rc = run_zero(S.flags + FLAG_BAR_COUNT, FLAG_WORDS - FLAG_BAR_COUNT, st)) != CASGD_OK)
        return rc;

    const int prec = opts ? opts->recur_prec : 0;
    const bool fp64 = prec == 64 || (prec == 0 && S.sb >= 512);
    const size_t lds = sparse_lds_bytes(S.sb, s, fp64 ? 8 : 4, P.Hp);
    const void* kern = fp64 ? reinterpret_cast<const void*>(k_sparse_fit<double>)
                            : reinterpret_cast<const void*>(k_sparse_fit<float>);
    if (lds > 65536) {
        if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
            hipSuccess) {
            (void)hipGetLastError();
            set_error("the sparse kernel needs %zu bytes of LDS per workgroup", lds);
            return CASGD_EUNSUPPORTED;
        }
    }
    int per_cu = 0;
    CASGD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kNT, lds));
    const int maxg = per_cu * device_cus();
    const int groups = (L + kLanesPerRecWG - 1) / kLanesPerRecWG;
    int grid = (opts && opts->grid_blocks > 0) ? opts->grid_blocks : device_cus();
    grid = std::min(grid, maxg);
    // Workgroups per lane group: a power of two dividing b; automatically 8
    // rows per workgroup (fewer workgroups if they would take more than half
    // of the grid).
    int K = 1;
    if (opts && opts->rec_split > 0) {
        K = opts->rec_split;
        if ((K & (K - 1)) != 0 || b % K != 0) {
            set_error("rec_split must be a power of two dividing b");
            return CASGD_EINVAL;
        }
    } else {
        while (b % (2 * K) == 0 && b / (2 * K) >= 8 && groups * 2 * K <= grid / 2) K *= 2;
    }
    int R = groups * K;
    if (grid <= R) {
        set_error("not enough resident workgroups (%d) for %d lanes", maxg, L);
        return CASGD_EUNSUPPORTED;
    }
    unsigned long long spin =
        (opts && opts->spin_limit > 0) ? (unsigned long long)opts->spin_limit : (1ull << 24);
    if (K > 1 && (rc = run_zero(reinterpret_cast<unsigned*>(S.pub), (int64_t)S.sb * L * 4, st)) !=
                     CASGD_OK)
        return rc;
    uint64_t h0 = outer_begin;
    int64_t Hn = n_outer;
    void* args[] = {&S, &h0, &Hn, &spin, &K, &R};
    CASGD_HIP(hipLaunchCooperativeKernel(kern, dim3(grid), dim3(kNT), args, (unsigned)lds, st));
    return CASGD_OK;
}

}  // namespace casgd

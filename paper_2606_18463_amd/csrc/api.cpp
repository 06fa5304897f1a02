// C ABI of libcasgd: argument validation, workspace layout and dispatch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#include <algorithm>

#include "internal.hpp"
#include "misc.hpp"
#include "recurrence.hpp"

namespace casgd {

// Per-thread message of the last failing call: a plain buffer, so that no
// destructor runs at thread or process exit.
static thread_local char t_err[512];

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(t_err, sizeof t_err, fmt, ap);
    va_end(ap);
}

casgd_status hip_fail(hipError_t e, const char* what) {
    set_error("%s failed: %s", what, hipGetErrorString(e));
    return CASGD_EDEVICE;
}

int dtype_bytes(int dt) {
    switch (dt) {
        case CASGD_F32: return 4;
        case CASGD_BF16: return 2;
        case CASGD_F16: return 2;
        case CASGD_FP8E4M3: return 1;
        default: return 0;
    }
}

int dtype_vec(int dt) { return 16 / dtype_bytes(dt); }
int slice_width_of(int dt) { return dtype_bytes(dt) ? kLPR * kEPL : 0; }

int device_cus() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    if (!cached[dev]) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cached[dev] = cus;
    }
    return cached[dev];
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

bool dense_layout(int64_t n, int dtype, int b, int s, DenseLayout* L) {
    const int sb = s * b;
    L->sb = sb;
    L->ts = (sb + kTile - 1) / kTile;
    L->ntiles = L->ts * (L->ts + 1) / 2;
    int needed = 0;
    for (int TJ = 0; TJ < L->ts; ++TJ)
        for (int TI = 0; TI <= TJ; ++TI) {
            const int rlast = std::min(TJ * kTile + kTile - 1, sb - 1);
            if ((TI * kTile) / b < rlast / b) ++needed;
        }
    L->needed = needed;
    {
        const int T = tiles128_per_side(sb);
        L->t128 = T * (T + 1) / 2;
        int n128 = 0;
        for (int TJ = 0; TJ < T; ++TJ)
            for (int TI = 0; TI <= TJ; ++TI) {
                const int rlast = std::min(TJ * kBig + kBig - 1, sb - 1);
                if ((TI * kBig) / b < rlast / b) ++n128;
            }
        L->n128 = n128;
    }
    L->bt = (b % kTile == 0) ? b / kTile : 0;
    L->gt = L->bt > 0 ? needed : L->ntiles;
    const int kstep = 4 * dtype_vec(dtype);
    const int64_t kpad = (n + kstep - 1) / kstep * kstep;
    // Row strides with a 256-byte pad: rows of the gathered block and of G are
    // read many at a time, and a power-of-two stride would put all of them on
    // one memory channel.
    L->ldy = (n + 127) / 128 * 128 + 256 / dtype_bytes(dtype);
    L->ldg = sb + 64;
    // Gram units: whole 64x64 tiles, or half tiles when there are fewer tiles
    // than compute units. K splits across workgroups (a power of two that
    // divides the eight XCDs) only for very small Gram matrices (units fill
    // less than a quarter of the chip), and while every wave keeps at least
    // max(128, 4 K steps) of K: the split-K handshake costs a cache
    // write-back per workgroup.
    const int ncu = device_cus();
    L->gna = L->gt < ncu ? 2 : 4;
    const int units = L->gna == 4 ? L->gt : 2 * L->gt;
    const int64_t kmin = std::max<int64_t>(128, 4 * kstep);
    int ksplit = 1;
    if (s > 1 && needed > 0)
        while (ksplit < 8 && 4 * units * ksplit < ncu && kpad / (2 * ksplit * 4) >= kmin)
            ksplit *= 2;
    int64_t kchunk = (kpad + ksplit - 1) / ksplit;
    kchunk = (kchunk + kstep - 1) / kstep * kstep;
    L->ksplit = ksplit;
    L->kchunk = kchunk;
    const int kw = slice_width_of(dtype);
    L->nslices = (int)((n + kw - 1) / kw);

    size_t off = 0;
    L->off_flags = off;
    off = align256(off + FLAG_WORDS * 4);
    L->off_tilecnt = off;
    off = align256(off + (size_t)L->ntiles * 2 * 4);
    const size_t gbytes = s > 1 ? (size_t)sb * L->ldg * 4 : 0;
    L->off_G0 = off;
    off = align256(off + gbytes);
    L->off_G1 = off;
    off = align256(off + gbytes);
    L->off_Gpart = off;
    if (s > 1 && L->ksplit > 1) off = align256(off + (size_t)L->ntiles * L->ksplit * 4096 * 4);
    L->off_rp0 = off;
    off = align256(off + (size_t)L->nslices * sb * 4);
    L->off_rp1 = off;
    off = align256(off + (size_t)L->nslices * sb * 4);
    L->off_c = off;
    off = align256(off + (size_t)sb * 4);
    L->off_r = off;
    off = align256(off + (size_t)sb * 4);
    L->off_pub = off;   // recurrence exchange: 2 * sb values of up to two words
    off = align256(off + (size_t)sb * 4 * sizeof(unsigned long long));
    const size_t sbpad = (size_t)(sb + 127) / 128 * 128;   // rows padded to whole 128-row tiles
    for (int k = 0; k < 3; ++k) {
        L->off_Y[k] = off;
        off = align256(off + sbpad * L->ldy * dtype_bytes(dtype));
        L->off_yI[k] = off;
        off = align256(off + (size_t)sb * 4);
        L->off_sI[k] = off;
        off = align256(off + (size_t)sb * 4);
    }
    L->total = off;
    // K-split region of the stand-alone 128-tile Gram (two workgroups per CU
    // resident): the tiles left after whole rounds of that many, split into
    // pieces of at least 16 K chunks of 128 bytes, at most 16 per tile; only
    // for rows of 64 chunks or more (with shorter rows the exchange costs
    // about as much as a piece: measured slower than whole tiles)
    {
        const int64_t nch = (n * dtype_bytes(dtype) + kChunkB - 1) / kChunkB;
        const int R = 2 * ncu, Tn = L->t128;
        const int rem = R <= 0 ? 0 : (Tn <= R ? Tn : Tn % R);
        int64_t S = 0;
        if (s > 1 && L->n128 > 0 && rem > 0 && nch >= 64)
            S = std::min<int64_t>({16, nch / 16, R / rem});
        L->sk_nslots = S >= 2 ? (int)(rem * S) : 0;
        L->total_sk = L->sk_nslots ? off + 256 + (size_t)L->sk_nslots * kGramSkWords * 8 : off;
    }
    return true;
}

void dense_bind(const DenseLayout& L, void* ws, size_t ws_bytes, Dense* P) {
    char* w = static_cast<char*>(ws);
    P->sb = L.sb;
    P->ts = L.ts;
    P->ntiles = L.ntiles;
    P->gt = L.gt;
    P->bt = L.bt;
    P->gna = L.gna;
    P->ksplit = L.ksplit;
    P->kchunk = L.kchunk;
    P->nslices = L.nslices;
    P->t128 = L.t128;
    P->g128 = 0;
    P->flags = reinterpret_cast<unsigned*>(w + L.off_flags);
    P->tile_cnt = reinterpret_cast<unsigned*>(w + L.off_tilecnt);
    P->G[0] = reinterpret_cast<float*>(w + L.off_G0);
    P->G[1] = reinterpret_cast<float*>(w + L.off_G1);
    P->Gpart = reinterpret_cast<float*>(w + L.off_Gpart);
    P->rp[0] = reinterpret_cast<float*>(w + L.off_rp0);
    P->rp[1] = reinterpret_cast<float*>(w + L.off_rp1);
    P->c = reinterpret_cast<float*>(w + L.off_c);
    P->r = reinterpret_cast<float*>(w + L.off_r);
    P->pub = reinterpret_cast<unsigned long long*>(w + L.off_pub);
    P->ldy = L.ldy;
    P->ldg = L.ldg;
    for (int k = 0; k < 3; ++k) {
        P->Y[k] = w + L.off_Y[k];
        P->yI[k] = reinterpret_cast<float*>(w + L.off_yI[k]);
        P->sI[k] = reinterpret_cast<float*>(w + L.off_sI[k]);
    }
    P->sk_nslots = 0;
    P->sk_epoch = nullptr;
    P->sk_slots = nullptr;
    if (L.sk_nslots && ws_bytes >= L.total_sk) {
        P->sk_nslots = L.sk_nslots;
        P->sk_epoch = reinterpret_cast<unsigned*>(w + L.total);
        P->sk_slots = reinterpret_cast<unsigned long long*>(w + L.total + 256);
    }
}

// ----------------------------------------------------------- validation

casgd_status check_bs(int32_t b, int32_t s) {
    if (b < 1 || s < 1) {
        set_error("b and s must be >= 1 (got b=%d, s=%d)", b, s);
        return CASGD_EINVAL;
    }
    if ((int64_t)b * s > 4096) {
        set_error("s*b = %lld exceeds the supported maximum 4096", (long long)b * s);
        return CASGD_EUNSUPPORTED;
    }
    return CASGD_OK;
}

casgd_status check_dense(const casgd_matrix* X) {
    if (!X) {
        set_error("X is NULL");
        return CASGD_EINVAL;
    }
    if (X->layout != CASGD_DENSE) {
        set_error("this entry point needs a dense X (layout %d)", X->layout);
        return CASGD_EUNSUPPORTED;
    }
    if (X->m < 1 || X->n < 1 || X->ld < X->n) {
        set_error("bad shape m=%lld n=%lld ld=%lld", (long long)X->m, (long long)X->n,
                  (long long)X->ld);
        return CASGD_EINVAL;
    }
    if (X->m > (1ll << 40) || X->n > (1ll << 31)) {
        set_error("shape m=%lld n=%lld too large", (long long)X->m, (long long)X->n);
        return CASGD_EUNSUPPORTED;
    }
    const int eb = dtype_bytes(X->dtype);
    if (!eb) {
        set_error("unknown dtype %d", X->dtype);
        return CASGD_EINVAL;
    }
    if (!X->values) {
        set_error("X->values is NULL");
        return CASGD_EINVAL;
    }
    if ((reinterpret_cast<uintptr_t>(X->values) & 15) || ((X->ld * eb) & 15)) {
        set_error("X must be 16-byte aligned with ld*elementsize a multiple of 16");
        return CASGD_EINVAL;
    }
    if (X->dtype == CASGD_FP8E4M3 && !X->row_scale) {
        set_error("FP8-E4M3 storage needs row_scale");
        return CASGD_EINVAL;
    }
    return CASGD_OK;
}

static casgd_status check_csr(const casgd_matrix* X) {
    if (!X || X->layout != CASGD_CSR) {
        set_error("expected a CSR matrix");
        return CASGD_EINVAL;
    }
    if (X->m < 1 || X->n < 1 || X->nnz < 0 || !X->row_ptr || (X->nnz > 0 && (!X->col_idx || !X->values))) {
        set_error("bad CSR matrix (m=%lld n=%lld nnz=%lld)", (long long)X->m, (long long)X->n,
                  (long long)X->nnz);
        return CASGD_EINVAL;
    }
    if (X->dtype != CASGD_F32) {
        set_error("CSR values must be FP32");
        return CASGD_EUNSUPPORTED;
    }
    if (X->n > (1ll << 31) - 1) {
        set_error("CSR column count too large");
        return CASGD_EUNSUPPORTED;
    }
    return CASGD_OK;
}

casgd_status check_loss(int loss) {
    if (loss != CASGD_LOSS_LOGISTIC && loss != CASGD_LOSS_LINEAR && loss != CASGD_LOSS_POISSON) {
        set_error("loss must be 0 (logistic), 1 (linear) or 2 (Poisson), got %d", loss);
        return CASGD_EINVAL;
    }
    return CASGD_OK;
}

static casgd_status check_scalars(double eta, double lambda) {
    if (!(eta > 0) || !std::isfinite(eta) || !(lambda >= 0) || !std::isfinite(lambda)) {
        set_error("need eta > 0 and lambda >= 0, both finite (eta=%g, lambda=%g)", eta, lambda);
        return CASGD_EINVAL;
    }
    return CASGD_OK;
}

casgd_status check_ws(const void* ws, size_t ws_bytes, size_t need) {
    if (!ws) {
        set_error("workspace is NULL");
        return CASGD_EINVAL;
    }
    if (reinterpret_cast<uintptr_t>(ws) & 255) {
        set_error("workspace must be 256-byte aligned");
        return CASGD_EINVAL;
    }
    if (ws_bytes < need) {
        set_error("workspace too small: %zu bytes given, %zu needed", ws_bytes, need);
        return CASGD_ENOMEM;
    }
    return CASGD_OK;
}

// Fill a Dense view for X, y, x and the scalars, bound to workspace ws.
casgd_status make_dense(const casgd_matrix* X, const float* y, float* x, double eta,
                               double lambda, int32_t b, int32_t s, uint64_t seed,
                               const casgd_opts* o, void* ws, size_t ws_bytes, Dense* P,
                               DenseLayout* L, bool need_ws) {
    casgd_status rc;
    if ((rc = check_dense(X)) != CASGD_OK) return rc;
    if ((rc = check_bs(b, s)) != CASGD_OK) return rc;
    if ((rc = check_scalars(eta, lambda)) != CASGD_OK) return rc;
    dense_layout(X->n, X->dtype, b, s, L);
    if (need_ws && (rc = check_ws(ws, ws_bytes, L->total)) != CASGD_OK) return rc;
    std::memset(P, 0, sizeof *P);
    P->X = X->values;
    P->scale = X->row_scale;
    P->y = y;
    P->x = x;
    P->m = X->m;
    P->n = X->n;
    P->ld = X->ld;
    P->b = b;
    P->s = s;
    P->seed = seed;
    P->alpha_d = eta / b;
    P->beta_d = 1.0 - eta * lambda;
    P->alpha = (float)P->alpha_d;
    P->beta = (float)P->beta_d;
    P->beta_s = (float)std::pow(P->beta_d, (double)s);
    if (need_ws) {
        dense_bind(*L, ws, ws_bytes, P);
    } else {
        P->sb = L->sb;
        P->ts = L->ts;
        P->ntiles = L->ntiles;
        P->ksplit = L->ksplit;
        P->kchunk = L->kchunk;
        P->nslices = L->nslices;
    }
    P->loss = o ? o->loss : CASGD_LOSS_LOGISTIC;
    if ((rc = check_loss(P->loss)) != CASGD_OK) return rc;
    P->e2e = o ? o->e2e : 0;
    if (P->e2e != 0) {
        const int want = P->e2e == 1 ? CASGD_BF16 : CASGD_F16;
        if (P->e2e != 1 && P->e2e != 2) {
            set_error("e2e must be 0, 1 (BF16) or 2 (FP16), got %d", P->e2e);
            return CASGD_EINVAL;
        }
        if (X->dtype != want) {
            set_error("e2e %s needs X stored in %s", P->e2e == 1 ? "BF16" : "FP16",
                      P->e2e == 1 ? "BF16" : "FP16");
            return CASGD_EINVAL;
        }
        if (o->recur_prec == 64) {
            set_error("e2e runs the corrections in FP32 (recur_prec 64 not allowed)");
            return CASGD_EINVAL;
        }
    }
    if (o && o->snapshot_every > 0) {
        if (!o->x_history) {
            set_error("snapshot_every > 0 needs x_history");
            return CASGD_EINVAL;
        }
        P->snap_every = o->snapshot_every;
        P->x_hist = o->x_history;
        P->t_hist = o->t_history;
    }
    if (o && o->phase_trace && o->phase_trace_outer > 0) {
        P->ptrace = o->phase_trace;
        P->ptrace_outer = o->phase_trace_outer;
    }
    return CASGD_OK;
}

}  // namespace casgd

using namespace casgd;

extern "C" {

const char* casgd_status_string(casgd_status st) {
    switch (st) {
        case CASGD_OK: return "ok";
        case CASGD_EINVAL: return "invalid argument";
        case CASGD_EUNSUPPORTED: return "unsupported";
        case CASGD_ENOMEM: return "workspace too small";
        case CASGD_EDEVICE: return "HIP runtime error";
        case CASGD_ENONFINITE: return "non-finite value";
        case CASGD_ETIMEOUT: return "grid barrier timeout";
        default: return "unknown status";
    }
}

const char* casgd_last_error(void) { return t_err; }

int32_t casgd_version(void) { return 100; }

casgd_status casgd_gram_workspace_size(const casgd_matrix* X, int32_t b, int32_t s,
                                       size_t* bytes) {
    casgd_status rc;
    if (!bytes) {
        set_error("bytes is NULL");
        return CASGD_EINVAL;
    }
    if ((rc = check_dense(X)) != CASGD_OK) return rc;
    if ((rc = check_bs(b, s)) != CASGD_OK) return rc;
    DenseLayout L;
    dense_layout(X->n, X->dtype, b, s, &L);
    *bytes = L.total_sk;
    return CASGD_OK;
}

casgd_status casgd_workspace_size(const casgd_matrix* X, int32_t b, int32_t s, size_t* bytes) {
    casgd_status rc;
    if (!bytes) {
        set_error("bytes is NULL");
        return CASGD_EINVAL;
    }
    if (X && X->layout == CASGD_CSR) return sparse_workspace_size(X, b, s, 1, bytes);
    if ((rc = check_dense(X)) != CASGD_OK) return rc;
    if ((rc = check_bs(b, s)) != CASGD_OK) return rc;
    DenseLayout L;
    dense_layout(X->n, X->dtype, b, s, &L);
    *bytes = L.total;
    return CASGD_OK;
}

casgd_status casgd_reset(void* ws, size_t ws_bytes, void* stream) {
    casgd_status rc;
    if ((rc = check_ws(ws, ws_bytes, FLAG_WORDS * 4)) != CASGD_OK) return rc;
    return run_zero(static_cast<unsigned*>(ws), FLAG_WORDS, (hipStream_t)stream);
}

casgd_status casgd_check(const void* ws, size_t ws_bytes, void* stream) {
    casgd_status rc;
    if ((rc = check_ws(ws, ws_bytes, FLAG_WORDS * 4)) != CASGD_OK) return rc;
    CASGD_HIP(hipStreamSynchronize((hipStream_t)stream));
    unsigned f[2] = {0, 0};
    CASGD_HIP(hipMemcpy(f, ws, sizeof f, hipMemcpyDeviceToHost));
    if (f[FLAG_TIMEOUT]) {
        set_error("a grid barrier of the fused kernel exceeded its spin limit");
        return CASGD_ETIMEOUT;
    }
    if (f[FLAG_NONFINITE]) {
        set_error("a margin, residual or weight became NaN or Inf");
        return CASGD_ENONFINITE;
    }
    unsigned ov = 0;
    CASGD_HIP(hipMemcpy(&ov, static_cast<const unsigned*>(ws) + 2, sizeof ov,
                        hipMemcpyDeviceToHost));
    if (ov) {
        set_error("a sparse tail-column bucket overflowed (results invalid)");
        return CASGD_EUNSUPPORTED;
    }
    return CASGD_OK;
}

casgd_status casgd_path_workspace_size(const casgd_matrix* X, int32_t b, int32_t s,
                                       int32_t lanes, size_t* bytes) {
    if (!bytes) {
        set_error("bytes is NULL");
        return CASGD_EINVAL;
    }
    if (X && X->layout == CASGD_CSR) return sparse_workspace_size(X, b, s, lanes, bytes);
    set_error("lambda lanes need a CSR X");
    return CASGD_EUNSUPPORTED;
}

casgd_status casgd_sparse_prepare(const casgd_matrix* X, int32_t b, int32_t s, int32_t lanes,
                                  void* ws, size_t ws_bytes, void* stream) {
    return sparse_prepare(X, b, s, lanes, ws, ws_bytes, stream);
}

casgd_status casgd_fit_path(const casgd_matrix* X, const float* y, float* x_lanes,
                            const double* lambdas, int32_t L, double eta, int32_t b, int32_t s,
                            uint64_t seed, uint64_t outer_begin, int64_t n_outer,
                            const casgd_opts* opts, void* ws, size_t ws_bytes, void* stream) {
    if (!X || X->layout != CASGD_CSR) {
        set_error("lambda lanes need a CSR X");
        return CASGD_EUNSUPPORTED;
    }
    return sparse_fit(X, y, x_lanes, lambdas, L, eta, b, s, seed, outer_begin, n_outer, opts, ws,
                      ws_bytes, stream);
}

casgd_status casgd_fit(const casgd_matrix* X, const float* y, float* x, double eta,
                       double lambda, int32_t b, int32_t s, uint64_t seed, uint64_t outer_begin,
                       int64_t n_outer, const casgd_opts* opts, void* ws, size_t ws_bytes,
                       void* stream) {
    if (X && X->layout == CASGD_CSR)
        return sparse_fit(X, y, x, &lambda, 1, eta, b, s, seed, outer_begin, n_outer, opts, ws,
                          ws_bytes, stream);
    if (!y || !x) {
        set_error("y and x must not be NULL");
        return CASGD_EINVAL;
    }
    if (n_outer < 0) {
        set_error("n_outer must be >= 0");
        return CASGD_EINVAL;
    }
    Dense P;
    DenseLayout L;
    casgd_status rc =
        make_dense(X, y, x, eta, lambda, b, s, seed, opts, ws, ws_bytes, &P, &L, true);
    if (rc != CASGD_OK) return rc;
    FitPlan plan;
    if ((rc = plan_fit(P, X->dtype, opts, n_outer, &plan)) != CASGD_OK) return rc;
    return run_fit(P, X->dtype, outer_begin, n_outer, plan, (hipStream_t)stream);
}

casgd_status casgd_step(const casgd_matrix* X, const float* y, float* x, double eta,
                        double lambda, int32_t b, int32_t s, uint64_t seed, uint64_t outer_iter,
                        const casgd_opts* opts, void* ws, size_t ws_bytes, void* stream) {
    return casgd_fit(X, y, x, eta, lambda, b, s, seed, outer_iter, 1, opts, ws, ws_bytes, stream);
}

static constexpr int kBatchMaxWG = 4096;

size_t casgd_batch_table_size(int32_t count) {
    if (count < 1) return 0;
    return align256((size_t)count * sizeof(Dense)) + (size_t)kBatchMaxWG * sizeof(int2);
}

// Cost model of one problem's fit on g workgroups: H outer iterations of a
// fixed part (the recurrence and the barriers) plus a parallel part (Gram
// flops and row traffic spread over the group). Rates per workgroup, from
// measurements on MI355X: the single-workgroup recurrence streams G_L at
// about 6 GB/s (320 us at b = 64, s = 16), the chain + helper form takes
// about 1.5 us per step plus two barriers.
static double batch_time(const Dense& P, int dtype, int variant, int g) {
    const double gl = 4.0 * P.b * (double)P.b * P.s * (P.s - 1) / 2.0;
    const double fixed = variant == 3 ? 1.5e-6 * P.s + 10e-6
                                      : (variant == 2 ? gl / 6e9 + 6e-6 : gl / 6e9 + 3e-6);
    const double flop_rate = dtype == CASGD_F32 ? 0.3e12 : 1.0e12;
    const double par = (double)P.s * (P.s - 1) * P.b * P.b * P.n / flop_rate +
                       3.0 * P.sb * (double)P.ldy * dtype_bytes(dtype) / 40e9;
    return (double)P.H * (fixed + par / g);
}

// Workgroups a variant needs at least: the recurrence group of variant 3
// (which also claims the Gram units when nobody else is there), one
// recurrence workgroup plus one Gram workgroup for variant 2, one otherwise.
static int batch_minimum(const Dense& P, int variant) {
    return variant == 3 ? 1 + rec_helpers(P.b, P.s) : (variant == 2 ? 2 : 1);
}

casgd_status casgd_fit_batch(casgd_problem* probs, int32_t count, int64_t spin_limit,
                             void* table, size_t table_bytes, void* stream) {
    if (!probs || count < 1) {
        set_error("need at least one problem");
        return CASGD_EINVAL;
    }
    const size_t need = casgd_batch_table_size(count);
    casgd_status rc;
    if ((rc = check_ws(table, table_bytes, need)) != CASGD_OK) return rc;
    const int dtype = probs[0].X.dtype;
    std::vector<Dense> D((size_t)count);
    std::vector<int> groups((size_t)count), minimum((size_t)count), variant((size_t)count);
    std::vector<char> autov((size_t)count, 0);
    size_t lds = 0;
    hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < count; ++i) {
        const casgd_problem& q = probs[i];
        if (q.X.dtype != dtype) {
            set_error("problem %d: all problems of a batch must share one storage dtype", i);
            return CASGD_EINVAL;
        }
        if (!q.y || !q.x || q.n_outer < 0) {
            set_error("problem %d: y and x must not be NULL and n_outer >= 0", i);
            return CASGD_EINVAL;
        }
        DenseLayout L;
        casgd_opts o;
        std::memset(&o, 0, sizeof o);
        o.recur_prec = q.recur_prec;
        o.fused_variant = q.variant;
        o.loss = q.loss;
        o.snapshot_every = q.snapshot_every;
        o.x_history = q.x_history;
        o.t_history = q.t_history;
        rc = make_dense(&q.X, q.y, q.x, q.eta, q.lambda, q.b, q.s, q.seed, &o, q.ws, q.ws_bytes,
                        &D[i], &L, true);
        if (rc != CASGD_OK) {
            std::string m = casgd_last_error();
            set_error("problem %d: %s", i, m.c_str());
            return rc;
        }
        FitPlan plan;
        if ((rc = plan_fit(D[i], dtype, &o, q.n_outer, &plan)) != CASGD_OK) return rc;
        D[i].h0 = q.outer_begin;
        D[i].H = q.n_outer;
        D[i].recur64 = plan.recur64;
        D[i].tpr = recurrence_tpr(kNT, q.b);
        variant[i] = plan.variant;
        autov[i] = q.variant == 0 && plan.variant == 3;
        lds = std::max(lds, fit_lds(D[i], dtype, plan.recur64));
        groups[i] = q.groups;
    }
    if (lds > 65536) {
        set_error("a problem of the batch needs more LDS than the fused kernel has");
        return CASGD_EUNSUPPORTED;
    }
    bool generic = false;   // some problem has another loss or end-to-end rounding
    for (int i = 0; i < count; ++i) generic = generic || D[i].loss != 0 || D[i].e2e != 0;
    const int maxg = std::min(batch_max_grid(dtype, lds, generic), kBatchMaxWG);
    // Automatic variant 3 needs its whole recurrence group resident: when the
    // groups do not fit, problems fall back to variant 2, those whose
    // modelled gain from variant 3 is smallest first.
    auto total_min = [&]() {
        int t = 0;
        for (int i = 0; i < count; ++i) t += groups[i] > 0 ? groups[i] : batch_minimum(D[i], variant[i]);
        return t;
    };
    while (total_min() > maxg) {
        int pick = -1;
        double best = 0.0;
        for (int i = 0; i < count; ++i) {
            if (!autov[i] || variant[i] != 3 || groups[i] > 0) continue;
            const int g3 = batch_minimum(D[i], 3);
            const double gain = batch_time(D[i], dtype, 2, g3) - batch_time(D[i], dtype, 3, g3);
            if (pick < 0 || gain < best) { pick = i; best = gain; }
        }
        if (pick < 0) break;
        variant[pick] = 2;
    }
    for (int i = 0; i < count; ++i) {
        D[i].variant = variant[i];
        minimum[i] = batch_minimum(D[i], variant[i]);
        if (groups[i] > 0 && groups[i] < minimum[i]) {
            set_error("problem %d: variant %d needs at least %d workgroups", i, variant[i],
                      minimum[i]);
            return CASGD_EINVAL;
        }
    }
    int fixed = 0, need_min = 0;
    for (int i = 0; i < count; ++i) {
        if (groups[i] > 0) fixed += groups[i];
        else need_min += minimum[i];
    }
    if (fixed + need_min > maxg) {
        set_error("batch needs %d workgroups, at most %d can be resident", fixed + need_min, maxg);
        return CASGD_EUNSUPPORTED;
    }
    // Automatic groups: start from the minimum and give each further
    // workgroup to the problem whose modelled finishing time is largest.
    for (int i = 0; i < count; ++i)
        if (groups[i] == 0) groups[i] = -minimum[i];
    int spare = maxg - fixed - need_min;
    while (spare > 0) {
        int worst = -1;
        double wt = -1.0;
        for (int i = 0; i < count; ++i) {
            if (groups[i] >= 0) continue;
            const double t = batch_time(D[i], dtype, variant[i], -groups[i]);
            if (t > wt) { wt = t; worst = i; }
        }
        if (worst < 0) break;
        const double gain = wt - batch_time(D[worst], dtype, variant[worst], -groups[worst] + 1);
        if (gain <= 1e-3 * wt) break;
        --groups[worst];
        --spare;
    }
    std::vector<int2> wgmap;
    for (int i = 0; i < count; ++i) {
        const int g = std::abs(groups[i]);
        D[i].gsize = g;
        const int nrec = variant[i] == 3 ? 1 + rec_helpers(D[i].b, D[i].s)
                                         : (variant[i] == 2 ? 1 : 0);
        D[i].g128 = choose_gram128(D[i], dtype, probs[i].gram_tile, std::max(1, g - nrec));
        for (int r = 0; r < g; ++r) wgmap.push_back(make_int2(i, r));
    }
    const int grid = (int)wgmap.size();
    for (int i = 0; i < count; ++i) {
        if ((rc = run_zero(D[i].tile_cnt, 2 * D[i].ntiles, st)) != CASGD_OK) return rc;
        if ((rc = run_zero(D[i].flags + FLAG_BAR_COUNT, FLAG_WORDS - FLAG_BAR_COUNT, st)) != CASGD_OK)
            return rc;
        if (D[i].variant == 3 &&
            (rc = run_zero(reinterpret_cast<unsigned*>(D[i].pub), (int64_t)D[i].sb * 8, st)) !=
                CASGD_OK)
            return rc;
    }
    char* tb = static_cast<char*>(table);
    Dense* tdev = reinterpret_cast<Dense*>(tb);
    int2* mdev = reinterpret_cast<int2*>(tb + align256((size_t)count * sizeof(Dense)));
    CASGD_HIP(hipMemcpyAsync(tdev, D.data(), D.size() * sizeof(Dense), hipMemcpyHostToDevice, st));
    CASGD_HIP(hipMemcpyAsync(mdev, wgmap.data(), wgmap.size() * sizeof(int2), hipMemcpyHostToDevice,
                             st));
    CASGD_HIP(hipStreamSynchronize(st));
    const unsigned long long spin = spin_limit > 0 ? (unsigned long long)spin_limit : (1ull << 24);
    if ((rc = run_fit_batch(tdev, mdev, grid, dtype, lds, spin, generic, st)) != CASGD_OK)
        return rc;
    for (int i = 0; i < count; ++i) {
        probs[i].groups = D[i].gsize;
        probs[i].variant = D[i].variant;
    }
    return CASGD_OK;
}

casgd_status casgd_sample_indices(uint64_t seed, uint64_t t0, int64_t count, int64_t m,
                                  int64_t* out, void* stream) {
    if (count < 0 || m < 1 || (count > 0 && !out)) {
        set_error("bad arguments (count=%lld, m=%lld)", (long long)count, (long long)m);
        return CASGD_EINVAL;
    }
    return run_sample(seed, t0, count, m, out, (hipStream_t)stream);
}

casgd_status casgd_gram_margin(const casgd_matrix* X, const float* x, int32_t b, int32_t s,
                               uint64_t seed, uint64_t outer_iter, float* G, float* r,
                               const casgd_opts* opts, void* ws, size_t ws_bytes, void* stream) {
    if (!G || (!x) != (!r)) {
        set_error("G must not be NULL, and x and r must both be given or both be NULL");
        return CASGD_EINVAL;
    }
    Dense P;
    DenseLayout L;
    casgd_status rc = make_dense(X, nullptr, const_cast<float*>(x), 1.0, 0.0, b, s, seed, nullptr,
                                 ws, ws_bytes, &P, &L, true);
    if (rc != CASGD_OK) return rc;
    P.ldg = P.sb;   // the caller's G is sb x sb
    const int gram_tile = opts ? opts->gram_tile : 0;
    if (gram_tile != 0 && gram_tile != 64 && gram_tile != 128) {
        set_error("gram_tile must be 0, 64 or 128 (got %d)", gram_tile);
        return CASGD_EINVAL;
    }
    // automatic: the K-split 128-tiles for long rows (128 chunks of 128 bytes
    // or more) when the workspace holds their region; otherwise the rule of
    // the fits
    const int64_t nch = (X->n * dtype_bytes(X->dtype) + kChunkB - 1) / kChunkB;
    P.g128 = (gram_tile == 0 && P.sk_nslots > 0 && nch >= 128) ||
             choose_gram128(P, X->dtype, gram_tile, device_cus());
    hipStream_t st = (hipStream_t)stream;
    if ((rc = run_zero(P.tile_cnt, 2 * P.ntiles, st)) != CASGD_OK) return rc;
    if ((rc = run_gather(P, X->dtype, outer_iter, st)) != CASGD_OK) return rc;
    if ((rc = run_gram(P, X->dtype, G, outer_iter, st)) != CASGD_OK) return rc;
    if (!x) return CASGD_OK;
    if ((rc = run_margin(P, X->dtype, outer_iter, P.rp[0], st)) != CASGD_OK) return rc;
    return run_margin_reduce(P, P.rp[0], outer_iter, r, st);
}

// Workspace of casgd_recurrence: the flag words, then the exchange words of
// the multi-workgroup form (2 * sb values of up to two 64-bit words).
static size_t rec_ws_pub_offset() { return align256((size_t)FLAG_WORDS * 4); }

size_t casgd_recurrence_workspace_size(int32_t b, int32_t s) {
    if (b < 1 || s < 1 || (int64_t)b * s > 4096) return 0;
    return rec_ws_pub_offset() + align256((size_t)b * s * 4 * sizeof(unsigned long long));
}

casgd_status casgd_recurrence(const float* G, const float* r, const float* yI, int32_t b,
                              int32_t s, double eta, double lambda, int32_t prec, int32_t loss,
                              int32_t form, float* c, float* delta, void* ws, size_t ws_bytes,
                              void* stream) {
    casgd_status rc;
    if ((s > 1 && !G) || !r || !yI || !c) {
        set_error("G, r, yI and c must not be NULL");
        return CASGD_EINVAL;
    }
    if ((rc = check_bs(b, s)) != CASGD_OK) return rc;
    if ((rc = check_scalars(eta, lambda)) != CASGD_OK) return rc;
    if ((rc = check_loss(loss)) != CASGD_OK) return rc;
    if (prec != 0 && prec != 32 && prec != 64) {
        set_error("prec must be 0, 32 or 64");
        return CASGD_EINVAL;
    }
    const bool multi_ok = (b == 16 || b == 32 || b == 64 || b == 128) && s > 1;
    if (form == 0) form = multi_ok ? 2 : 1;
    if (form != 1 && form != 2) {
        set_error("form must be 0, 1 or 2 (got %d)", form);
        return CASGD_EINVAL;
    }
    if (form == 2 && !multi_ok) {
        set_error("form 2 needs b = 16, 32, 64 or 128 and s > 1");
        return CASGD_EUNSUPPORTED;
    }
    if ((form == 2 || ws) &&
        (rc = check_ws(ws, ws_bytes, casgd_recurrence_workspace_size(b, s))) != CASGD_OK)
        return rc;
    Dense P;
    std::memset(&P, 0, sizeof P);
    P.b = b;
    P.s = s;
    P.sb = b * s;
    P.ldg = P.sb;
    P.alpha_d = eta / b;
    P.beta_d = 1.0 - eta * lambda;
    P.alpha = (float)P.alpha_d;
    P.beta = (float)P.beta_d;
    P.m = 1;
    P.loss = loss;
    if (ws) {
        P.flags = static_cast<unsigned*>(ws);
        P.pub = reinterpret_cast<unsigned long long*>(static_cast<char*>(ws) + rec_ws_pub_offset());
    }
    const bool fp64 = prec == 64 || (prec == 0 && P.sb >= 512);
    hipStream_t st = (hipStream_t)stream;
    if (form == 1) return run_recurrence(P, G, nullptr, 0, r, yI, c, delta, fp64, st);
    // the exchange words start from zero (the chain workgroup clears them when done)
    if ((rc = run_zero(reinterpret_cast<unsigned*>(P.pub), (int64_t)P.sb * 8, st)) != CASGD_OK)
        return rc;
    return run_recurrence_multi(P, G, r, yI, c, delta, fp64, 1ull << 24, st);
}

casgd_status casgd_update(const casgd_matrix* X, float* x, const float* c, int32_t b, int32_t s,
                          uint64_t seed, uint64_t outer_iter, double eta, double lambda, void* ws,
                          size_t ws_bytes, void* stream) {
    if (!x || !c) {
        set_error("x and c must not be NULL");
        return CASGD_EINVAL;
    }
    Dense P;
    DenseLayout L;
    casgd_status rc =
        make_dense(X, nullptr, x, eta, lambda, b, s, seed, nullptr, ws, ws_bytes, &P, &L, true);
    if (rc != CASGD_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    if ((rc = run_gather(P, X->dtype, outer_iter, st)) != CASGD_OK) return rc;
    return run_update(P, X->dtype, c, outer_iter, st);
}

casgd_status casgd_quantize(const float* src, int64_t m, int64_t n, int64_t ld_src, int32_t dtype,
                            void* dst, int64_t ld_dst, float* row_scale, void* stream) {
    const int eb = dtype_bytes(dtype);
    if (!src || !dst || m < 1 || n < 1 || ld_src < n || ld_dst < n || !eb) {
        set_error("bad arguments to casgd_quantize");
        return CASGD_EINVAL;
    }
    if (dtype == CASGD_FP8E4M3 && !row_scale) {
        set_error("FP8-E4M3 needs row_scale");
        return CASGD_EINVAL;
    }
    return run_quantize(src, m, n, ld_src, dtype, dst, ld_dst, row_scale, nullptr,
                        (hipStream_t)stream);
}

casgd_status casgd_quantize_scaled(const float* src, int64_t m, int64_t n, int64_t ld_src,
                                   const float* col_scale, int32_t dtype, void* dst, int64_t ld_dst,
                                   float* row_scale, void* stream) {
    const int eb = dtype_bytes(dtype);
    if (!src || !dst || !col_scale || m < 1 || n < 1 || ld_src < n || ld_dst < n || !eb) {
        set_error("bad arguments to casgd_quantize_scaled");
        return CASGD_EINVAL;
    }
    if (dtype == CASGD_FP8E4M3 && !row_scale) {
        set_error("FP8-E4M3 needs row_scale");
        return CASGD_EINVAL;
    }
    return run_quantize(src, m, n, ld_src, dtype, dst, ld_dst, row_scale, col_scale,
                        (hipStream_t)stream);
}

casgd_status casgd_mlp_features(const float* stats, int64_t N, const float* norm, float* feats,
                                void* stream) {
    if (N < 0 || (N > 0 && (!stats || !norm || !feats))) {
        set_error("bad arguments to casgd_mlp_features");
        return CASGD_EINVAL;
    }
    return run_mlp_features(stats, N, norm, feats, (hipStream_t)stream);
}

casgd_status casgd_mlp_forward(const float* params, const float* feats, int64_t N, float* out,
                               float* pre, void* stream) {
    if (N < 0 || !params || (N > 0 && (!feats || !out))) {
        set_error("bad arguments to casgd_mlp_forward");
        return CASGD_EINVAL;
    }
    return run_mlp_forward(params, feats, N, out, pre, (hipStream_t)stream);
}

size_t casgd_mlp_workspace_size(int64_t N, int32_t P) {
    return align256(mlp_loss_ws(P > 0 ? P : 1)) + align256(mlp_backward_ws(N));
}

casgd_status casgd_mlp_loss_grad(const float* out, const int64_t* seg_off, int32_t P, int64_t N,
                                 const float* t_d, const float* t_eta, float w_eta, double* loss,
                                 float* g_out, void* ws, size_t ws_bytes, void* stream) {
    casgd_status rc;
    if (!out || !seg_off || P < 1 || N < 1 || !t_d || !t_eta || !loss || !g_out) {
        set_error("bad arguments to casgd_mlp_loss_grad");
        return CASGD_EINVAL;
    }
    if ((rc = check_ws(ws, ws_bytes, casgd_mlp_workspace_size(N, P))) != CASGD_OK) return rc;
    return run_mlp_loss_grad(out, seg_off, P, N, t_d, t_eta, w_eta, loss, g_out,
                             static_cast<double*>(ws), (hipStream_t)stream);
}

casgd_status casgd_mlp_backward(const float* params, const float* feats, const float* pre,
                                const float* g_out, int64_t N, int32_t P, float* grad, void* ws,
                                size_t ws_bytes, void* stream) {
    casgd_status rc;
    if (!params || !grad || N < 0 || (N > 0 && (!feats || !pre || !g_out))) {
        set_error("bad arguments to casgd_mlp_backward");
        return CASGD_EINVAL;
    }
    if ((rc = check_ws(ws, ws_bytes, casgd_mlp_workspace_size(N, P))) != CASGD_OK) return rc;
    float* partial = reinterpret_cast<float*>(static_cast<char*>(ws) +
                                              align256(mlp_loss_ws(P > 0 ? P : 1)));
    return run_mlp_backward(params, feats, pre, g_out, N, grad, partial, (hipStream_t)stream);
}

casgd_status casgd_adam_step(float* params, const float* grad, float* m1, float* m2,
                             int32_t count, int64_t t, float lr, float beta1, float beta2,
                             float eps, void* stream) {
    if (!params || !grad || !m1 || !m2 || count < 1 || t < 1) {
        set_error("bad arguments to casgd_adam_step");
        return CASGD_EINVAL;
    }
    return run_adam(params, grad, m1, m2, count, t, lr, beta1, beta2, eps, (hipStream_t)stream);
}

casgd_status casgd_mlp_feature_norm(const float* stats, int64_t N, float* norm, void* stream) {
    if (N < 1 || !stats || !norm) {
        set_error("bad arguments to casgd_mlp_feature_norm");
        return CASGD_EINVAL;
    }
    return run_feature_norm(stats, N, norm, (hipStream_t)stream);
}

casgd_status casgd_mlp_apply(const float* out, int64_t N, float* q, float* eta, void* stream) {
    if (N < 1 || !out || !q || !eta) {
        set_error("bad arguments to casgd_mlp_apply");
        return CASGD_EINVAL;
    }
    return run_mlp_apply(out, N, q, eta, (hipStream_t)stream);
}

casgd_status casgd_jacobi_target(const float* hdiag, int64_t n, float* t_d, float* q,
                                 void* stream) {
    if (n < 1 || !hdiag || !t_d) {
        set_error("bad arguments to casgd_jacobi_target");
        return CASGD_EINVAL;
    }
    return run_jacobi_target(hdiag, n, t_d, q, (hipStream_t)stream);
}

size_t casgd_hess_diag_workspace_size(const casgd_matrix* X) {
    return X ? hess_ws(X) : 0;
}

casgd_status casgd_hess_diag(const casgd_matrix* X, const float* x, double lambda, float* hdiag,
                             void* ws, size_t ws_bytes, void* stream) {
    casgd_status rc;
    if (!x || !hdiag) {
        set_error("x and hdiag must not be NULL");
        return CASGD_EINVAL;
    }
    if ((rc = check_dense(X)) != CASGD_OK) return rc;
    if ((rc = check_ws(ws, ws_bytes, hess_ws(X))) != CASGD_OK) return rc;
    return run_hess_diag(X, x, lambda, hdiag, ws, (hipStream_t)stream);
}

size_t casgd_logloss_workspace_size(int64_t count) {
    return count > 0 ? (size_t)count * kLossBlocks * sizeof(double) : 0;
}

casgd_status casgd_loss(const casgd_matrix* X, const float* y, const float* xs, int64_t count,
                        int64_t x_stride, int32_t loss, double* out, void* ws, size_t ws_bytes,
                        void* stream) {
    if (!X || !y || !xs || !out || count < 1 || x_stride < X->n) {
        set_error("bad arguments to casgd_loss");
        return CASGD_EINVAL;
    }
    casgd_status rc;
    if ((rc = check_loss(loss)) != CASGD_OK) return rc;
    if (X->layout == CASGD_DENSE && (rc = check_dense(X)) != CASGD_OK) return rc;
    if (X->layout == CASGD_CSR && (rc = check_csr(X)) != CASGD_OK) return rc;
    if ((rc = check_ws(ws, ws_bytes, casgd_logloss_workspace_size(count))) != CASGD_OK) return rc;
    return run_loss(X, y, xs, count, x_stride, loss, out, static_cast<double*>(ws),
                    (hipStream_t)stream);
}

casgd_status casgd_logloss(const casgd_matrix* X, const float* y, const float* xs, int64_t count,
                           int64_t x_stride, double* out, void* ws, size_t ws_bytes,
                           void* stream) {
    return casgd_loss(X, y, xs, count, x_stride, CASGD_LOSS_LOGISTIC, out, ws, ws_bytes, stream);
}

size_t casgd_colstats_workspace_size(const casgd_matrix* X) {
    if (!X || X->n < 1) return 0;
    return (size_t)kStatRowBlocks * X->n * 4 * sizeof(double);
}

casgd_status casgd_colstats(const casgd_matrix* X, float* stats, void* ws, size_t ws_bytes,
                            void* stream) {
    if (!X || !stats) {
        set_error("X and stats must not be NULL");
        return CASGD_EINVAL;
    }
    casgd_status rc;
    if (X->layout == CASGD_DENSE && (rc = check_dense(X)) != CASGD_OK) return rc;
    if (X->layout == CASGD_CSR && (rc = check_csr(X)) != CASGD_OK) return rc;
    if ((rc = check_ws(ws, ws_bytes, casgd_colstats_workspace_size(X))) != CASGD_OK) return rc;
    return run_colstats(X, stats, static_cast<double*>(ws), (hipStream_t)stream);
}

}  // extern "C"

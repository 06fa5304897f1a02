// Thm. 5.1 (mixed-precision local error of one outer iteration) evaluated at
// run time and used to choose the storage format of X and the precision of
// the inner corrections.
//
// The sampled block of one outer iteration is gathered, its strict
// block-lower Gram matrix and margins are formed and the exact (lambda = 0,
// the theorem's setting) residual history d is run on the GPU with the
// library's kernels; the source quantities of the theorem are then
// evaluated on the host in FP64:
//   ||Y||_2, K_s = ||(I - L_sigma alpha |G_L|)^{-1}||_2, ||H_L||_2   (Lanczos)
//   T_g = || |Y|^T |d| ||,  T_r = || |Y| |x| ||,  T_G = || H_L |d| ||,
//   T_c = (sum_j (j b ||G_{j,0:j-1}||_F ||d_{0:j-1}||)^2)^(1/2),
// with H_{j,i} = |Y_j| |Y_i|^T (i < j). With one device the two all-reduce
// slots vanish. Each slot's coefficient multiplies its unit roundoff (or
// Higham factor); candidate assignments are tried from the cheapest storage
// format up and the first whose bound (1 + C_loc Omega) sum E stays within
// the caller's relative budget (and inside the theorem's validity domain,
// Omega <= 1/2) is chosen.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace casgd {
namespace {

constexpr double kU32 = 5.9604644775390625e-08;   // 2^-24
constexpr double kU64 = 1.1102230246251565e-16;   // 2^-53
constexpr double kUBF16 = 0.00390625;             // 2^-8
constexpr double kUF16 = 0.00048828125;           // 2^-11
constexpr double kUFP8 = 0.0625;                  // 2^-4 (E4M3: 3 mantissa bits)

double gamma_q(double q, double u) {
    const double qu = q * u;
    return qu < 1.0 ? qu / (1.0 - qu) : INFINITY;
}

double dot(const std::vector<double>& a, const std::vector<double>& b) {
    double s = 0.0;
    for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
    return s;
}

// Largest eigenvalue of a symmetric tridiagonal matrix (diagonal a, off
// diagonal e) by bisection on the Sturm count.
double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& e) {
    const size_t k = a.size();
    double lo = INFINITY, hi = -INFINITY;
    for (size_t i = 0; i < k; ++i) {
        const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(e[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    // number of eigenvalues below x
    auto below = [&](double x) {
        int cnt = 0;
        double q = a[0] - x;
        if (q < 0) ++cnt;
        for (size_t i = 1; i < k; ++i) {
            const double qq = q != 0.0 ? q : 1e-300;
            q = a[i] - x - e[i - 1] * e[i - 1] / qq;
            if (q < 0) ++cnt;
        }
        return cnt;
    };
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (below(mid) >= (int)k) hi = mid;
        else lo = mid;
    }
    return hi;
}

// Largest eigenvalue of a symmetric positive semidefinite operator of
// dimension dim (Lanczos with full reorthogonalisation, start vector from
// a fixed SplitMix64 stream).
template <class Op>
double lanczos_max(int64_t dim, Op apply, int kmax) {
    kmax = (int)std::min<int64_t>(kmax, dim);
    std::vector<std::vector<double>> V;
    std::vector<double> al, be;
    std::vector<double> v((size_t)dim);
    uint64_t z = 0x5eedull;
    for (auto& vi : v) {
        z += 0x9e3779b97f4a7c15ull;
        uint64_t t = z;
        t = (t ^ (t >> 30)) * 0xbf58476d1ce4e5b9ull;
        t = (t ^ (t >> 27)) * 0x94d049bb133111ebull;
        t ^= t >> 31;
        vi = 0.5 + (double)(t >> 11) * 0x1.0p-53;   // positive start: overlaps the Perron vector
    }
    double nv = std::sqrt(dot(v, v));
    for (auto& vi : v) vi /= nv;
    V.push_back(v);
    double last = 0.0;
    for (int k = 0; k < kmax; ++k) {
        std::vector<double> w = apply(V[k]);
        const double a = dot(w, V[k]);
        al.push_back(a);
        for (int pass = 0; pass < 2; ++pass)
            for (const auto& q : V) {
                const double c = dot(w, q);
                for (size_t i = 0; i < w.size(); ++i) w[i] -= c * q[i];
            }
        const double b = std::sqrt(dot(w, w));
        const double est = tridiag_max_eig(al, be);
        if (b <= 1e-13 * std::max(1e-300, std::fabs(est))) return est;
        if (k >= 8 && std::fabs(est - last) <= 1e-14 * std::fabs(est)) return est;
        last = est;
        be.push_back(b);
        for (auto& wi : w) wi /= b;
        V.push_back(std::move(w));
    }
    return tridiag_max_eig(al, std::vector<double>(be.begin(), be.begin() + (al.size() - 1)));
}

}  // namespace
}  // namespace casgd

using namespace casgd;

extern "C" size_t casgd_precision_workspace_size(const casgd_matrix* X, int32_t b, int32_t s) {
    size_t need = 0;
    if (casgd_workspace_size(X, b, s, &need) != CASGD_OK) return 0;
    const size_t sb = (size_t)b * s;
    // dense workspace, then G (sb x sb), r, delta, c (FP32) and the
    // recurrence's flag words
    return ((need + 255) & ~(size_t)255) + ((sb * sb * 4 + 255) & ~(size_t)255) +
           3 * ((sb * 4 + 255) & ~(size_t)255) + 4096;
}

extern "C" casgd_status casgd_select_precision(const casgd_matrix* X, const float* y, const float* x,
                                               double eta, int32_t b, int32_t s, uint64_t seed,
                                               uint64_t outer_iter, int32_t loss,
                                               double rel_budget, uint32_t allowed,
                                               casgd_precision_report* out, void* ws,
                                               size_t ws_bytes, void* stream) {
    casgd_status rc;
    if (!X || !y || !x || !out) {
        set_error("X, y, x and out must not be NULL");
        return CASGD_EINVAL;
    }
    if ((rc = check_dense(X)) != CASGD_OK) return rc;
    if (X->dtype != CASGD_F32) {
        set_error("casgd_select_precision reads the FP32 master copy of X (dtype CASGD_F32)");
        return CASGD_EINVAL;
    }
    if ((rc = check_loss(loss)) != CASGD_OK) return rc;
    if (!(rel_budget > 0) || !std::isfinite(rel_budget)) {
        set_error("rel_budget must be positive and finite");
        return CASGD_EINVAL;
    }
    if ((rc = check_ws(ws, ws_bytes, casgd_precision_workspace_size(X, b, s))) != CASGD_OK)
        return rc;
    Dense P;
    DenseLayout L;
    if ((rc = make_dense(X, y, const_cast<float*>(x), eta, 0.0, b, s, seed, nullptr, ws, ws_bytes,
                         &P, &L, true)) != CASGD_OK)
        return rc;
    const int64_t sb = (int64_t)s * b, n = X->n;
    char* base = static_cast<char*>(ws) + ((L.total + 255) & ~(size_t)255);
    float* G = reinterpret_cast<float*>(base);
    base += ((size_t)sb * sb * 4 + 255) & ~(size_t)255;
    float* r = reinterpret_cast<float*>(base);
    base += ((size_t)sb * 4 + 255) & ~(size_t)255;
    float* dlt = reinterpret_cast<float*>(base);
    base += ((size_t)sb * 4 + 255) & ~(size_t)255;
    float* cc = reinterpret_cast<float*>(base);
    hipStream_t st = (hipStream_t)stream;

    // GPU: gather, Gram + margins, the lambda = 0 corrections in FP64
    P.ldg = sb;
    if ((rc = run_zero(P.tile_cnt, 2 * P.ntiles, st)) != CASGD_OK) return rc;
    if ((rc = run_gather(P, CASGD_F32, outer_iter, st)) != CASGD_OK) return rc;
    if (s > 1 && (rc = run_gram(P, CASGD_F32, G, outer_iter, st)) != CASGD_OK) return rc;
    if ((rc = run_margin(P, CASGD_F32, outer_iter, P.rp[0], st)) != CASGD_OK) return rc;
    if ((rc = run_margin_reduce(P, P.rp[0], outer_iter, r, st)) != CASGD_OK) return rc;
    const int slot = slot_of_host(outer_iter);
    if ((rc = casgd_recurrence(G, r, P.yI[slot], b, s, eta, 0.0, 64, loss, 1, cc, dlt, nullptr, 0,
                               stream)) != CASGD_OK)
        return rc;
    // host copies (a planning call: synchronous)
    std::vector<float> Yf((size_t)sb * P.ldy), Gf(s > 1 ? (size_t)sb * sb : 1), rf(sb), df(sb),
        xf(n);
    CASGD_HIP(hipStreamSynchronize(st));
    CASGD_HIP(hipMemcpy(Yf.data(), P.Y[slot], Yf.size() * 4, hipMemcpyDeviceToHost));
    if (s > 1) CASGD_HIP(hipMemcpy(Gf.data(), G, Gf.size() * 4, hipMemcpyDeviceToHost));
    CASGD_HIP(hipMemcpy(rf.data(), r, sb * 4, hipMemcpyDeviceToHost));
    CASGD_HIP(hipMemcpy(df.data(), dlt, sb * 4, hipMemcpyDeviceToHost));
    CASGD_HIP(hipMemcpy(xf.data(), x, n * 4, hipMemcpyDeviceToHost));

    const double alpha = eta / b;
    auto blk = [&](int64_t t) { return t / b; };
    auto Yat = [&](int64_t t, int64_t k) { return (double)Yf[(size_t)t * P.ldy + k]; };
    auto GL = [&](int64_t t, int64_t u) {
        return blk(u) < blk(t) ? (double)Gf[(size_t)t * sb + u] : 0.0;
    };
    std::vector<double> d(sb), ad(sb), z(sb);
    for (int64_t t = 0; t < sb; ++t) {
        d[t] = df[t];
        ad[t] = std::fabs(d[t]);
    }
    // margins of the exact recurrence (for the Poisson Lipschitz constant)
    for (int64_t t = 0; t < sb; ++t) {
        double a = 0.0;
        for (int64_t u = 0; u < blk(t) * b; ++u) a += GL(t, u) * d[u];
        z[t] = rf[t] + alpha * a;
    }
    double L_sigma = 0.25, D_delta = 1.0;
    if (loss == CASGD_LOSS_LINEAR) L_sigma = 1.0;
    if (loss == CASGD_LOSS_POISSON) {
        double zm = -INFINITY;
        for (double v : z) zm = std::max(zm, v);
        L_sigma = std::exp(zm);
    }
    if (loss != CASGD_LOSS_LOGISTIC) {
        D_delta = 0.0;
        for (double v : ad) D_delta = std::max(D_delta, v);
    }
    // ||Y||_2 from the smaller Gram side
    double normY;
    if (sb <= n) {
        normY = std::sqrt(lanczos_max(sb, [&](const std::vector<double>& v) {
            std::vector<double> w(n, 0.0), o(sb, 0.0);
            for (int64_t t = 0; t < sb; ++t)
                for (int64_t k = 0; k < n; ++k) w[k] += Yat(t, k) * v[t];
            for (int64_t t = 0; t < sb; ++t) {
                double a = 0.0;
                for (int64_t k = 0; k < n; ++k) a += Yat(t, k) * w[k];
                o[t] = a;
            }
            return o;
        }, 160));
    } else {
        normY = std::sqrt(lanczos_max(n, [&](const std::vector<double>& v) {
            std::vector<double> w(sb, 0.0), o(n, 0.0);
            for (int64_t t = 0; t < sb; ++t) {
                double a = 0.0;
                for (int64_t k = 0; k < n; ++k) a += Yat(t, k) * v[k];
                w[t] = a;
            }
            for (int64_t t = 0; t < sb; ++t)
                for (int64_t k = 0; k < n; ++k) o[k] += Yat(t, k) * w[t];
            return o;
        }, 160));
    }
    // K_s: N = (I - M)^{-1}, M = L_sigma alpha |G_L| (strictly block-lower,
    // so N v is a forward substitution over blocks and N^T v a backward one)
    auto Nv = [&](const std::vector<double>& v) {
        std::vector<double> o(v);
        for (int64_t t = 0; t < sb; ++t) {
            double a = 0.0;
            for (int64_t u = 0; u < blk(t) * b; ++u) a += std::fabs(GL(t, u)) * o[u];
            o[t] += L_sigma * alpha * a;
        }
        return o;
    };
    auto NTv = [&](const std::vector<double>& v) {
        std::vector<double> o(v);
        for (int64_t u = sb - 1; u >= 0; --u) {
            double a = 0.0;
            for (int64_t t = (blk(u) + 1) * b; t < sb; ++t) a += std::fabs(GL(t, u)) * o[t];
            o[u] += L_sigma * alpha * a;
        }
        return o;
    };
    const double K_s = s > 1 ? std::sqrt(lanczos_max(sb, [&](const std::vector<double>& v) {
        return NTv(Nv(v));
    }, 160)) : 1.0;
    // H_L v via prefix sums over blocks of |Y|^T v; H_L^T v via suffix sums
    auto HLv = [&](const std::vector<double>& v) {
        std::vector<double> o(sb, 0.0), pre(n, 0.0);
        for (int j = 0; j < s; ++j) {
            for (int64_t t = (int64_t)j * b; t < (int64_t)(j + 1) * b; ++t) {
                double a = 0.0;
                for (int64_t k = 0; k < n; ++k) a += std::fabs(Yat(t, k)) * pre[k];
                o[t] = a;
            }
            for (int64_t t = (int64_t)j * b; t < (int64_t)(j + 1) * b; ++t)
                for (int64_t k = 0; k < n; ++k) pre[k] += std::fabs(Yat(t, k)) * v[t];
        }
        return o;
    };
    auto HLTv = [&](const std::vector<double>& v) {
        std::vector<double> o(sb, 0.0), suf(n, 0.0);
        for (int j = s - 1; j >= 0; --j) {
            for (int64_t t = (int64_t)j * b; t < (int64_t)(j + 1) * b; ++t) {
                double a = 0.0;
                for (int64_t k = 0; k < n; ++k) a += std::fabs(Yat(t, k)) * suf[k];
                o[t] = a;
            }
            for (int64_t t = (int64_t)j * b; t < (int64_t)(j + 1) * b; ++t)
                for (int64_t k = 0; k < n; ++k) suf[k] += std::fabs(Yat(t, k)) * v[t];
        }
        return o;
    };
    const double normHL = s > 1 ? std::sqrt(lanczos_max(sb, [&](const std::vector<double>& v) {
        return HLTv(HLv(v));
    }, 160)) : 0.0;
    // source quantities
    double Tg = 0.0, Tr = 0.0, TG = 0.0, Tc = 0.0, nYtd = 0.0, nxs = 0.0;
    {
        std::vector<double> g(n, 0.0), ytd(n, 0.0);
        for (int64_t t = 0; t < sb; ++t)
            for (int64_t k = 0; k < n; ++k) {
                g[k] += std::fabs(Yat(t, k)) * ad[t];
                ytd[k] += Yat(t, k) * d[t];
            }
        for (int64_t k = 0; k < n; ++k) {
            Tg += g[k] * g[k];
            nYtd += ytd[k] * ytd[k];
            const double xs = (double)xf[k] + alpha * ytd[k];
            nxs += xs * xs;
        }
        Tg = std::sqrt(Tg);
        nYtd = std::sqrt(nYtd);
        nxs = std::sqrt(nxs);
        for (int64_t t = 0; t < sb; ++t) {
            double a = 0.0;
            for (int64_t k = 0; k < n; ++k) a += std::fabs(Yat(t, k)) * std::fabs((double)xf[k]);
            Tr += a * a;
        }
        Tr = std::sqrt(Tr);
        const std::vector<double> h = HLv(ad);
        for (double v : h) TG += v * v;
        TG = std::sqrt(TG);
        double dpre = 0.0;
        for (int j = 1; j < s; ++j) {
            for (int64_t u = (int64_t)(j - 1) * b; u < (int64_t)j * b; ++u) dpre += d[u] * d[u];
            double gf = 0.0;
            for (int64_t t = (int64_t)j * b; t < (int64_t)(j + 1) * b; ++t)
                for (int64_t u = 0; u < (int64_t)j * b; ++u) gf += GL(t, u) * GL(t, u);
            const double term = (double)j * b * std::sqrt(gf) * std::sqrt(dpre);
            Tc += term * term;
        }
        Tc = std::sqrt(Tc);
    }
    std::memset(out, 0, sizeof *out);
    out->alpha = alpha;
    out->norm_Y = normY;
    out->K_s = K_s;
    out->norm_HL = normHL;
    out->T_g = Tg;
    out->T_r = Tr;
    out->T_G = TG;
    out->T_c = Tc;
    out->norm_x_next = nxs;
    out->L_sigma = L_sigma;
    out->D_delta = D_delta;
    const double a1 = alpha * normY * K_s * L_sigma;
    // per-slot coefficients (E_slot = coef * unit roundoff or Higham factor)
    out->coef[CASGD_SLOT_A] = a1 * Tr + 2 * alpha * a1 * TG + alpha * Tg;
    out->coef[CASGD_SLOT_R] = a1 * Tr;
    out->coef[CASGD_SLOT_G] = alpha * a1 * TG;
    out->coef[CASGD_SLOT_C] = a1 * Tr + 2 * alpha * a1 * TG + alpha * a1 * Tc;
    out->coef[CASGD_SLOT_SIGMA] = alpha * normY * K_s * 8.0 * D_delta * std::sqrt((double)sb);
    out->coef[CASGD_SLOT_GRAD] = alpha * Tg;
    out->coef[CASGD_SLOT_X] = nxs + alpha * nYtd;
    // candidates, cheapest first: storage FP8, BF16, FP16, FP32; corrections
    // FP32 before FP64
    double maxabs = 0.0;
    for (int64_t t = 0; t < sb; ++t)
        for (int64_t k = 0; k < n; ++k) maxabs = std::max(maxabs, std::fabs(Yat(t, k)));
    const int order[4] = {CASGD_FP8E4M3, CASGD_BF16, CASGD_F16, CASGD_F32};
    const double uA_of[4] = {0.0, kUBF16, kUF16, kUFP8};   // indexed by dtype
    if (allowed == 0) allowed = 0xF;
    out->chosen = -1;
    int k = 0;
    for (int oi = 0; oi < 4; ++oi) {
        const int dt = order[oi];
        if (!(allowed & (1u << dt))) continue;
        if (dt == CASGD_F16 && maxabs >= 65504.0) continue;   // outside the FP16 range
        for (int rp = 0; rp < 2; ++rp) {
            casgd_precision_candidate& c = out->cand[k++];
            const double uA = uA_of[dt];
            const double uc = rp == 0 ? kU32 : kU64;
            c.dtype = dt;
            c.recur_prec = rp == 0 ? 32 : 64;
            c.u[CASGD_SLOT_A] = uA;
            c.u[CASGD_SLOT_R] = (dt == CASGD_F32 ? 0.0 : 2 * uA) + gamma_q((double)n, kU32);
            c.u[CASGD_SLOT_G] = c.u[CASGD_SLOT_R];
            c.u[CASGD_SLOT_C] = uc;
            c.u[CASGD_SLOT_SIGMA] = uc;
            c.u[CASGD_SLOT_GRAD] = (dt == CASGD_F32 ? 0.0 : 2 * uA) + gamma_q((double)sb, kU32);
            c.u[CASGD_SLOT_X] = kU32;
            double sum = 0.0;
            for (int q = 0; q < CASGD_SLOTS; ++q) {
                c.E[q] = out->coef[q] * c.u[q];
                sum += c.E[q];
            }
            const double omega = std::max({uA, c.u[CASGD_SLOT_R], gamma_q((double)(s - 1) * b, uc),
                                           c.u[CASGD_SLOT_GRAD], uc, kU32});
            const double tau = K_s * L_sigma * alpha * (2 * uA + c.u[CASGD_SLOT_G]) * normHL;
            c.Omega = std::max(omega, tau);
            c.sum = sum;
            c.bound = (1.0 + 2.0 * c.Omega) * sum;
            c.rel_bound = nxs > 0 ? c.bound / nxs : INFINITY;
            c.valid = c.Omega <= 0.5 && (double)(s - 1) * b * uc < 1.0 && std::isfinite(c.bound);
            if (out->chosen < 0 && c.valid && c.rel_bound <= rel_budget) out->chosen = k - 1;
        }
    }
    out->ncand = k;
    if (out->chosen < 0) {
        // nothing meets the budget: the most accurate valid assignment
        for (int i = k - 1; i >= 0; --i)
            if (out->cand[i].valid) {
                out->chosen = i;
                break;
            }
        out->meets_budget = 0;
    } else {
        out->meets_budget = 1;
    }
    if (out->chosen < 0) {
        set_error("no precision assignment satisfies the theorem's validity conditions");
        return CASGD_EUNSUPPORTED;
    }
    out->dtype = out->cand[out->chosen].dtype;
    out->recur_prec = out->cand[out->chosen].recur_prec;
    return CASGD_OK;
}

// Sparse (CSR) s-step SGD with lambda lanes: device structures and phases.
//
// Columns are split once per (X, b, s) into a head (the most frequent columns,
// at most kHeadMax) and a tail. For every outer iteration the sampled rows are
// gathered into
//   * a dense FP32 head panel Yh (rows x Hp), whose Gram is computed with the
//     same MFMA tile routine as the dense path, and
//   * per-row tail lists (column, value).
// Tail columns are appended to per-column buckets; the owner of G row t then
// adds v_t v_u for every bucket entry u of an earlier block, visiting its own
// columns in order, so every G entry is accumulated in a fixed order.
// L lanes (regularisation strengths) share the samples, the gathered rows
// and G; only margins, residuals, c and x are per lane (x is n x L).
#pragma once

#include "recurrence.hpp"

namespace casgd {

constexpr int kHeadMax = 512;     // dense head columns at most
constexpr int kBucketCap = 64;    // tail bucket capacity per column and outer iteration
constexpr int kMaxLanes = 64;
constexpr int kLanesPerRecWG = 4; // lanes per recurrence workgroup

enum : int { FLAG_OVERFLOW = 2 };  // a tail bucket exceeded its capacity

struct Sparse {
    const int64_t* rp;
    const int32_t* ci;
    const float* va;
    const float* y;
    float* x;               // n x L, lane fastest
    int64_t m, n;
    int L;
    int b, s, sb;
    uint64_t seed;
    double alpha_d;
    const double* lbeta;    // L: 1 - eta*lambda_l
    const float* lbs;       // L: beta_l^s
    const int32_t* head_id; // n: head index or -1
    const int32_t* head_col;// H
    int H, Hp;              // head columns, padded to a multiple of 128
    int maxlen;             // longest row of X
    unsigned* flags;
    // per slot h % 3
    float* Yh[3];           // sbpad x Hp
    int32_t* tcol[3];       // sb x maxlen
    float* tval[3];         // sb x maxlen
    int32_t* tlen[3];       // sb
    float* yI[3];           // sb
    // per outer-iteration parity h % 2
    unsigned* bcnt[2];      // n
    int2* bent[2];          // n x kBucketCap of (t, value bits)
    float* G[2];
    float* r;               // sb x L
    float* c;               // sb x L
    float* x_hist;
    int64_t* t_hist;
    int64_t snap_every;
    unsigned long long* pub;  // delta exchange of the recurrence: 2 words per (row, lane)
    int64_t* ptrace;        // phase clock (8 words per outer iteration) or nullptr
    int64_t ptrace_outer;
    Dense gram;             // view for the head-panel Gram (MFMA tiles)
};

template <typename T>
__device__ __forceinline__ T spick3(const T (&a)[3], int k) {
    return k == 0 ? a[0] : (k == 1 ? a[1] : a[2]);
}
// Orders this wave's LDS accesses (a wave-scope barrier for scratch that only
// the wave uses).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

template <typename T>
__device__ __forceinline__ T spick2(const T (&a)[2], int k) {
    return k == 0 ? a[0] : a[1];
}

// Gather row t of outer h: one wave per row. The head panel row is built in
// LDS (`hrow`, Hp floats per wave) and written out whole; tail entries keep
// their column order (compacted with a wave ballot).
__device__ __forceinline__ void sparse_gather(const Sparse& S, uint64_t h, int wave_id,
                                              int nwaves, float* hrow) {
    const int lane = threadIdx.x & 63;
    const int slot = slot_of(h);
    float* Yh = spick3(S.Yh, slot);
    int32_t* tcol = spick3(S.tcol, slot);
    float* tval = spick3(S.tval, slot);
    int32_t* tlen = spick3(S.tlen, slot);
    float* yI = spick3(S.yI, slot);
    const int sbpad = (S.sb + kTile - 1) / kTile * kTile;
    const uint64_t t0 = h * (uint64_t)S.sb;
    for (int t = wave_id; t < sbpad; t += nwaves) {
        for (int q = lane; q < S.Hp; q += 64) hrow[q] = 0.f;
        __builtin_amdgcn_wave_barrier();
        if (t < S.sb) {
            const int64_t row = sample_row(S.seed, t0 + t, S.m);
            const int64_t p0 = S.rp[row], p1 = S.rp[row + 1];
            int ntail = 0;
            for (int64_t p = p0; p < p1; p += 64) {
                const int64_t pp = p + lane;
                const bool ok = pp < p1;
                const int col = ok ? S.ci[pp] : 0;
                const float v = ok ? S.va[pp] : 0.f;
                const int hid = ok ? S.head_id[col] : -1;
                if (ok && hid >= 0) hrow[hid] = v;
                const bool tail = ok && hid < 0;
                const uint64_t mask = __ballot(tail);
                const int before = __popcll(mask & ((1ull << lane) - 1ull));
                if (tail) {
                    tcol[(int64_t)t * S.maxlen + ntail + before] = col;
                    tval[(int64_t)t * S.maxlen + ntail + before] = v;
                }
                ntail += __popcll(mask);
            }
            if (lane == 0) {
                tlen[t] = ntail;
                yI[t] = S.y[row];
            }
        }
        __builtin_amdgcn_wave_barrier();
        for (int q = lane; q < S.Hp; q += 64) Yh[(int64_t)t * S.Hp + q] = hrow[q];
        __builtin_amdgcn_wave_barrier();
    }
}

// Append every tail entry of outer h to its column's bucket (parity h % 2).
__device__ __forceinline__ void sparse_bucket(const Sparse& S, uint64_t h, int gtid, int nthreads) {
    const int slot = slot_of(h);
    const int32_t* tcol = spick3(S.tcol, slot);
    const float* tval = spick3(S.tval, slot);
    const int32_t* tlen = spick3(S.tlen, slot);
    unsigned* bcnt = spick2(S.bcnt, (int)(h & 1));
    int2* bent = spick2(S.bent, (int)(h & 1));
    const int64_t total = (int64_t)S.sb * S.maxlen;
    for (int64_t e = gtid; e < total; e += nthreads) {
        const int t = (int)(e / S.maxlen), k = (int)(e - (int64_t)t * S.maxlen);
        if (k >= tlen[t]) continue;
        const int col = tcol[e];
        const unsigned pos = atomicAdd(bcnt + col, 1u);
        if (pos < (unsigned)kBucketCap)
            bent[(int64_t)col * kBucketCap + pos] = make_int2(t, __float_as_int(tval[e]));
        else
            raise_flag(S.flags, FLAG_OVERFLOW);
    }
}

// Tail part of the Gram of outer h: the owner thread of row t adds
// v_t v_u into G[t][u] for each of its tail columns (in column order) and each
// bucket entry u of an earlier block. Must run after the head-panel Gram.
__device__ __forceinline__ void sparse_gram_tail(const Sparse& S, uint64_t h, float* G, int gtid,
                                                 int nthreads) {
    const int slot = slot_of(h);
    const int32_t* tcol = spick3(S.tcol, slot);
    const float* tval = spick3(S.tval, slot);
    const int32_t* tlen = spick3(S.tlen, slot);
    const unsigned* bcnt = spick2(S.bcnt, (int)(h & 1));
    const int2* bent = spick2(S.bent, (int)(h & 1));
    for (int t = gtid; t < S.sb; t += nthreads) {
        const int bt = t / S.b;
        if (bt == 0) continue;
        const int nt = tlen[t];
        for (int k = 0; k < nt; ++k) {
            const int col = tcol[(int64_t)t * S.maxlen + k];
            const float vt = tval[(int64_t)t * S.maxlen + k];
            const int cnt = min((int)bcnt[col], kBucketCap);
            const int2* be = bent + (int64_t)col * kBucketCap;
            for (int q = 0; q < cnt; ++q) {
                const int2 e = be[q];
                if (e.x / S.b < bt) G[(int64_t)t * S.sb + e.x] += vt * __int_as_float(e.y);
            }
        }
    }
}

// Margins of outer h for all lanes. One wave per (16 rows, 16 lanes) tile:
// the head part R = Yh Xh (rows x H times H x lanes) with FP32 MFMA
// 16x16x4, then each lane adds the tail entries of its four outputs' rows.
// Output layout of the 16x16 MFMA: lane q, register v hold row 4*(q/16)+v,
// column q%16 of the tile.
__device__ __forceinline__ void sparse_margins(const Sparse& S, uint64_t h, int wave_id,
                                               int nwaves) {
    const int lane = threadIdx.x & 63;
    const int slot = slot_of(h);
    const float* Yh = spick3(S.Yh, slot);
    const int32_t* tcol = spick3(S.tcol, slot);
    const float* tval = spick3(S.tval, slot);
    const int32_t* tlen = spick3(S.tlen, slot);
    const int L = S.L;
    const int rt = (S.sb + 15) / 16, lt = (L + 15) / 16;
    const int li = lane & 15, lg = lane >> 4;
    for (int item = wave_id; item < rt * lt; item += nwaves) {
        const int t0 = (item / lt) * 16, l0 = (item % lt) * 16;
        v4f acc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = v4f{0.f, 0.f, 0.f, 0.f};
        const int jl = l0 + li;
        const bool lok = jl < L;
        // A[i][k] = Yh[t0+i][hc0+k] (lane: i = li, k = lg); B[k][j] = x[head_col[hc0+k]][l0+j]
        const float* arow = Yh + (int64_t)(t0 + li) * S.Hp;
        for (int hc0 = 0; hc0 < S.H; hc0 += 16) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int hc = hc0 + 4 * k + lg;
                const float a = arow[hc];
                const float bv = (hc < S.H && lok) ? S.x[(int64_t)S.head_col[hc] * L + jl] : 0.f;
                acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc[k], 0, 0, 0);
            }
        }
        v4f d = acc[0] + acc[1] + acc[2] + acc[3];
        if (lok) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int t = t0 + 4 * lg + v;
                if (t >= S.sb) continue;
                float r = d[v];
                const int nt = tlen[t];
                for (int k = 0; k < nt; ++k)
                    r = fmaf(tval[(int64_t)t * S.maxlen + k],
                             S.x[(int64_t)tcol[(int64_t)t * S.maxlen + k] * L + jl], r);
                S.r[(int64_t)t * L + jl] = r;
            }
        }
    }
}

// Update of outer h for all lanes: x <- beta^s x + alpha * Y^T c.
//  * head columns: one wave per (16 head columns, 16 lanes) tile computes
//    Yh^T c (H x rows times rows x lanes) with FP32 MFMA 16x16x4;
//  * tail columns present in the block: one wave per column sums its bucket
//    in increasing t for every lane (see below);
//  * all other columns: x <- beta^s x.
__device__ __forceinline__ void sparse_update(const Sparse& S, uint64_t h, int wave_id, int nwaves,
                                              int gtid, int nthreads, int64_t snap_row,
                                              int2* sorted) {
    const int lane = threadIdx.x & 63;
    const int slot = slot_of(h);
    const float* Yh = spick3(S.Yh, slot);
    const int32_t* tcol = spick3(S.tcol, slot);
    const int32_t* tlen = spick3(S.tlen, slot);
    const unsigned* bcnt = spick2(S.bcnt, (int)(h & 1));
    const int2* bent = spick2(S.bent, (int)(h & 1));
    const int L = S.L;
    const float alpha = (float)S.alpha_d;
    const int li = lane & 15, lg = lane >> 4;
    // head columns: D[i][j] = sum_t Yh[t][hc0+i] c[t][l0+j]
    const int ht = (S.H + 15) / 16, lt = (L + 15) / 16;
    for (int item = wave_id; item < ht * lt; item += nwaves) {
        const int hc0 = (item / lt) * 16, l0 = (item % lt) * 16;
        const int jl = l0 + li;
        const bool lok = jl < L;
        v4f acc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = v4f{0.f, 0.f, 0.f, 0.f};
        for (int t0 = 0; t0 < S.sb; t0 += 16) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int t = t0 + 4 * k + lg;
                const float a = Yh[(int64_t)t * S.Hp + hc0 + li];  // padded rows are zero
                const float bv = (t < S.sb && lok) ? S.c[(int64_t)t * L + jl] : 0.f;
                acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bv, acc[k], 0, 0, 0);
            }
        }
        const v4f g = acc[0] + acc[1] + acc[2] + acc[3];
        if (lok) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int hc = hc0 + 4 * lg + v;
                if (hc >= S.H) continue;
                const int64_t k = S.head_col[hc];
                const float xn = S.lbs[jl] * S.x[k * L + jl] + alpha * g[v];
                S.x[k * L + jl] = xn;
                if (!isfinite(xn)) raise_flag(S.flags, FLAG_NONFINITE);
                if (snap_row >= 0) S.x_hist[(snap_row * S.n + k) * L + jl] = xn;
            }
        }
    }
    // Tail columns of the block. The owner of a column is its bucket entry
    // with the smallest t; each wave scans 64 entries at a time, and for each
    // owner among them the whole wave handles the column: lane q ranks bucket
    // entry q by t (the t of a column's entries are distinct) and stores it
    // at its rank in the wave's LDS scratch, then lane l (one per lambda lane)
    // adds the entries in increasing t, four loads in flight at a time.
    const int64_t total = (int64_t)S.sb * S.maxlen;
    for (int64_t e0 = (int64_t)wave_id * 64; e0 < total; e0 += (int64_t)nwaves * 64) {
        const int64_t e = e0 + lane;
        bool own = false;
        int col = 0;
        if (e < total) {
            const int t = (int)(e / S.maxlen), kk = (int)(e - (int64_t)t * S.maxlen);
            if (kk < tlen[t]) {
                col = tcol[e];
                const int cnt = min((int)bcnt[col], kBucketCap);
                const int2* be = bent + (int64_t)col * kBucketCap;
                int tmin = t;
                for (int q = 0; q < cnt; ++q) tmin = min(tmin, be[q].x);
                own = tmin == t;
            }
        }
        unsigned long long mask = __ballot(own);
        while (mask) {
            const int src = __ffsll((unsigned long long)mask) - 1;
            mask &= mask - 1;
            const int ccol = __shfl(col, src, kWave);
            const int cnt = min((int)bcnt[ccol], kBucketCap);
            const int2 en = lane < cnt ? bent[(int64_t)ccol * kBucketCap + lane]
                                       : make_int2(0x7fffffff, 0);
            int rank = 0;
            for (int q = 0; q < cnt; ++q) {
                const int tq = __shfl(en.x, q, kWave);
                rank += (tq < en.x || (tq == en.x && q < lane)) ? 1 : 0;
            }
            wave_lds_sync();
            if (lane < cnt) sorted[rank] = en;
            wave_lds_sync();
            const int l = lane;
            if (l < L) {
                float g = 0.f;
                int p = 0;
                for (; p + 4 <= cnt; p += 4) {
                    const int2 e0v = sorted[p], e1v = sorted[p + 1], e2v = sorted[p + 2],
                               e3v = sorted[p + 3];
                    const float c0 = S.c[(int64_t)e0v.x * L + l], c1 = S.c[(int64_t)e1v.x * L + l],
                                c2 = S.c[(int64_t)e2v.x * L + l], c3 = S.c[(int64_t)e3v.x * L + l];
                    g = fmaf(__int_as_float(e0v.y), c0, g);
                    g = fmaf(__int_as_float(e1v.y), c1, g);
                    g = fmaf(__int_as_float(e2v.y), c2, g);
                    g = fmaf(__int_as_float(e3v.y), c3, g);
                }
                for (; p < cnt; ++p) {
                    const int2 ev = sorted[p];
                    g = fmaf(__int_as_float(ev.y), S.c[(int64_t)ev.x * L + l], g);
                }
                const float xn = S.lbs[l] * S.x[(int64_t)ccol * L + l] + alpha * g;
                S.x[(int64_t)ccol * L + l] = xn;
                if (!isfinite(xn)) raise_flag(S.flags, FLAG_NONFINITE);
                if (snap_row >= 0) S.x_hist[(snap_row * S.n + ccol) * L + l] = xn;
            }
        }
    }
    // untouched columns: decay only
    for (int64_t q = gtid; q < S.n * L; q += nthreads) {
        const int64_t k = q / L;
        const int l = (int)(q - k * L);
        if (S.head_id[k] >= 0 || bcnt[k] != 0u) continue;
        const float xn = S.lbs[l] * S.x[q];
        S.x[q] = xn;
        if (snap_row >= 0) S.x_hist[snap_row * S.n * L + q] = xn;
    }
}

// Clear the bucket counts of outer h (every tail entry clears its column).
__device__ __forceinline__ void sparse_clear_buckets(const Sparse& S, uint64_t h, int gtid,
                                                     int nthreads) {
    const int slot = slot_of(h);
    const int32_t* tcol = spick3(S.tcol, slot);
    const int32_t* tlen = spick3(S.tlen, slot);
    unsigned* bcnt = spick2(S.bcnt, (int)(h & 1));
    const int64_t total = (int64_t)S.sb * S.maxlen;
    for (int64_t e = gtid; e < total; e += nthreads) {
        const int t = (int)(e / S.maxlen), kk = (int)(e - (int64_t)t * S.maxlen);
        if (kk < tlen[t]) bcnt[tcol[e]] = 0u;
    }
}

// Residual corrections for lanes [l0, l0 + nl), nl <= kLanesPerRecWG, by the
// K workgroups of one lane group; workgroup k of the group owns rows
// [k b/K, (k+1) b/K) of every row block. In step j each computes z_j and
// delta_j of its own rows (every 16-byte piece of a G row prefix is loaded
// once and applied to all lanes of the group), publishes the deltas as tagged
// words and collects those of the other rows before step j + 1. The owner of
// a word clears it after the grid barrier that follows the recurrence, so
// every outer iteration starts from cleared words.
// LDS: dl (sb x kLanesPerRecWG ACC), pw (kLanesPerRecWG x (s+1) ACC).
template <typename ACC, int NT>
__device__ __forceinline__ void sparse_recurrence(const Sparse& S, const float* G, uint64_t h,
                                                  int l0, int nl, int k, int K, ACC* dl, ACC* pw,
                                                  unsigned long long spin) {
    constexpr int NL = kLanesPerRecWG;
    const int tid = threadIdx.x;
    const int b = S.b, s = S.s, sb = S.sb, L = S.L;
    const int RB = b / K, q_lo = k * RB;
    // threads per row: a power of two, at most one wave
    int TPR = 1;
    while (TPR < 64 && 2 * TPR * RB <= NT) TPR *= 2;
    const int RPP = NT / TPR;
    const int sub = tid % TPR;
    if (tid < NL) {
        ACC p = 1;
        const ACC be = tid < nl ? (ACC)S.lbeta[l0 + tid] : (ACC)1;
        for (int q = 0; q <= s; ++q) { pw[tid * (s + 1) + q] = p; p *= be; }
    }
    __syncthreads();
    const ACC alpha = (ACC)S.alpha_d;
    const float* yI = spick3(S.yI, slot_of(h));
    for (int j = 0; j < s; ++j) {
        const int nv = (j * b) >> 2;   // 16-byte pieces of the row prefix
        for (int q0 = 0; q0 < RB; q0 += RPP) {
            const int q = q0 + tid / TPR;
            const bool active = q < RB;
            const int t = j * b + q_lo + min(q, RB - 1);
            ACC acc[NL];
#pragma unroll
            for (int l = 0; l < NL; ++l) acc[l] = 0;
            const float4* g4 = reinterpret_cast<const float4*>(G + (int64_t)t * sb);
            for (int base = sub; base < nv; base += kRB * TPR) {
                float4 g[kRB];
#pragma unroll
                for (int u = 0; u < kRB; ++u) g[u] = g4[min(base + u * TPR, nv - 1)];
#pragma unroll
                for (int u = 0; u < kRB; ++u) {
                    const int v = base + u * TPR;
                    if (v < nv) {
                        const int e = 4 * v;
                        const int i = e / b;
                        const ACC* d = dl + e * NL;
#pragma unroll
                        for (int l = 0; l < NL; ++l) {
                            const ACC part = (ACC)g[u].x * d[l] + (ACC)g[u].y * d[NL + l] +
                                             (ACC)g[u].z * d[2 * NL + l] +
                                             (ACC)g[u].w * d[3 * NL + l];
                            acc[l] += pw[l * (s + 1) + (j - 1 - i)] * part;
                        }
                    }
                }
            }
#pragma unroll
            for (int l = 0; l < NL; ++l) acc[l] = group_sum_rt(acc[l], TPR);
            if (active && sub == 0) {
                const ACC yv = (ACC)yI[t];
#pragma unroll
                for (int l = 0; l < NL; ++l) {
                    if (l < nl) {
                        const ACC r = (ACC)S.r[(int64_t)t * L + l0 + l];
                        const ACC z = pw[l * (s + 1) + j] * r + alpha * acc[l];
                        const ACC d = yv / ((ACC)1 + exp(yv * z));
                        if (!isfinite(z)) raise_flag(S.flags, FLAG_NONFINITE);
                        dl[t * NL + l] = d;
                        S.c[(int64_t)t * L + l0 + l] = (float)(pw[l * (s + 1) + (s - 1 - j)] * d);
                        if (K > 1 && j + 1 < s) pub_put(S.pub + 2 * ((int64_t)t * L + l0 + l), d);
                    } else {
                        dl[t * NL + l] = 0;
                    }
                }
            }
        }
        if (K > 1 && j + 1 < s) {
            // deltas of the rows the other workgroups of the group own
            for (int w = tid; w < b * NL; w += NT) {
                const int q = w / NL, l = w - q * NL;
                if (q >= q_lo && q < q_lo + RB) continue;
                const int t = j * b + q;
                ACC d = 0;
                if (l < nl) pub_wait(S.pub + 2 * ((int64_t)t * L + l0 + l), d, S.flags, spin);
                dl[t * NL + l] = d;
            }
        }
        __syncthreads();
    }
}

// Clears the exchange words of the rows a recurrence workgroup owns (after
// the grid barrier that ends the recurrence).
__device__ __forceinline__ void sparse_pub_clear(const Sparse& S, int l0, int nl, int k, int K) {
    if (K <= 1) return;
    const int b = S.b, RB = b / K, n = (S.s - 1) * RB * nl;
    for (int w = threadIdx.x; w < n; w += blockDim.x) {
        const int l = w % nl, rq = w / nl, j = rq / RB, q = rq - j * RB;
        const int64_t t = (int64_t)j * b + k * RB + q;
        unsigned long long* p = S.pub + 2 * (t * S.L + l0 + l);
        __hip_atomic_store(p, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(p + 1, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace casgd

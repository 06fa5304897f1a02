// Sparse (CSR) s-step SGD with lambda lanes: device structures and phases.
//
// Columns are split once per (X, b, s) into a head (the most frequent columns,
// at most kHeadMax) and a tail. For every outer iteration the sampled rows are
// gathered into
//   * a dense FP32 head panel Yh (rows x Hp), whose Gram is computed with the
//     same MFMA tile routine as the dense path, and
//   * per-row tail lists (column, value).
// Tail columns are appended to per-column buckets; the wave that owns G row t
// then adds v_t v_u for every bucket entry u of an earlier block, visiting
// the row's columns in order, so every G entry is accumulated in a fixed
// order.
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
    int32_t* tlist[2];      // n: the distinct tail columns of the block, in arrival order
    unsigned* tlcnt;        // 2: their number, per parity
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
    int loss;               // LOSS_* (residual formula of the recurrence)
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

// Append every tail entry of outer h to its column's bucket (parity h % 2);
// the first entry of a column also appends the column to the tail list.
__device__ __forceinline__ void sparse_bucket(const Sparse& S, uint64_t h, int gtid, int nthreads) {
    const int slot = slot_of(h);
    const int32_t* tcol = spick3(S.tcol, slot);
    const float* tval = spick3(S.tval, slot);
    const int32_t* tlen = spick3(S.tlen, slot);
    unsigned* bcnt = spick2(S.bcnt, (int)(h & 1));
    int2* bent = spick2(S.bent, (int)(h & 1));
    const int64_t total = (int64_t)S.sb * S.maxlen;
    const int lane = threadIdx.x & 63;
    // wave-uniform loop: new columns are appended to the tail list with one
    // counter atomic per wave
    for (int64_t e0 = gtid - lane; e0 < total; e0 += nthreads) {
        const int64_t e = e0 + lane;
        bool ok = e < total;
        int t = 0, col = 0;
        unsigned pos = 1u;
        if (ok) {
            t = (int)(e / S.maxlen);
            const int k = (int)(e - (int64_t)t * S.maxlen);
            ok = k < tlen[t];
        }
        if (ok) {
            col = tcol[e];
            pos = atomicAdd(bcnt + col, 1u);
            if (pos < (unsigned)kBucketCap)
                bent[(int64_t)col * kBucketCap + pos] = make_int2(t, __float_as_int(tval[e]));
            else
                raise_flag(S.flags, FLAG_OVERFLOW);
        }
        const unsigned long long first = __ballot(ok && pos == 0u);
        if (first) {
            unsigned base = 0;
            if (lane == __ffsll((unsigned long long)first) - 1)
                base = atomicAdd(S.tlcnt + (h & 1), (unsigned)__popcll(first));
            base = __shfl(base, __ffsll((unsigned long long)first) - 1, kWave);
            if (ok && pos == 0u) {
                const unsigned ix = base + (unsigned)__popcll(first & ((1ull << lane) - 1ull));
                if (ix < (unsigned)S.n) spick2(S.tlist, (int)(h & 1))[ix] = col;
                else raise_flag(S.flags, FLAG_OVERFLOW);
            }
        }
    }
}

// Tail part of the Gram of outer h: one wave per row t of blocks 1.. . It
// visits the row's tail columns in column order; for each, the lanes take the
// column's bucket entries u of earlier blocks (distinct rows, so no two lanes
// touch the same u) and add v_t v_u into a row buffer in LDS (`rowbuf`, sb
// floats of this wave). The buffer is then added to G row t. Every G entry is
// thus accumulated in a fixed order. Must run after the head-panel Gram.
__device__ __forceinline__ void sparse_gram_tail(const Sparse& S, uint64_t h, float* G,
                                                 int wave_id, int nwaves, float* rowbuf) {
    const int lane = threadIdx.x & 63;
    const int slot = slot_of(h);
    const int32_t* tcol = spick3(S.tcol, slot);
    const float* tval = spick3(S.tval, slot);
    const int32_t* tlen = spick3(S.tlen, slot);
    const unsigned* bcnt = spick2(S.bcnt, (int)(h & 1));
    const int2* bent = spick2(S.bent, (int)(h & 1));
    const int ql = min(lane, kBucketCap - 1);
    for (int t = S.b + wave_id; t < S.sb; t += nwaves) {
        const int nt = tlen[t];
        if (nt == 0) continue;
        const int pre = (t / S.b) * S.b;   // columns of earlier blocks
        for (int u = lane; u < pre; u += 64) rowbuf[u] = 0.f;
        wave_lds_sync();
        for (int k0 = 0; k0 < nt; k0 += 64) {
            const int kn = min(64, nt - k0);
            const int64_t ek = (int64_t)t * S.maxlen + k0 + min(lane, kn - 1);
            const int col = tcol[ek];
            const float vt = tval[ek];
            const int cnt = min((int)bcnt[col], kBucketCap);
            // entry of the next column, loaded one step ahead
            int2 nxt = bent[(int64_t)__shfl(col, 0, kWave) * kBucketCap + ql];
            for (int k = 0; k < kn; ++k) {
                const int2 e = nxt;
                const float v = __shfl(vt, k, kWave);
                const int c = __shfl(cnt, k, kWave);
                const int kk = min(k + 1, kn - 1);
                nxt = bent[(int64_t)__shfl(col, kk, kWave) * kBucketCap + ql];
                if (lane < c && e.x < pre) rowbuf[e.x] += v * __int_as_float(e.y);
                wave_lds_sync();
            }
        }
        float* grow = G + (int64_t)t * S.sb;
        for (int u = lane; u < pre; u += 64) {
            const float v = rowbuf[u];
            if (v != 0.f) grow[u] += v;
        }
        wave_lds_sync();
    }
}

// Margins of outer h for all lanes. One workgroup per (16 rows, 16 lanes)
// tile: the head part R = Yh Xh (rows x H times H x lanes) with FP32 MFMA
// 16x16x4, wave w taking the 16-column chunks w, w + 4, ... (four chunks of
// loads in flight), the partial tiles added in wave order through LDS (`red`,
// 4 KB); then thread (i, j) of the tile adds the tail entries of row i in
// column order, eight loads in flight. Output layout of the 16x16 MFMA: lane
// q, register v hold row 4*(q/16)+v, column q%16 of the tile.
__device__ __forceinline__ void sparse_margins(const Sparse& S, uint64_t h, float* red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = slot_of(h);
    const float* Yh = spick3(S.Yh, slot);
    const int32_t* tcol = spick3(S.tcol, slot);
    const float* tval = spick3(S.tval, slot);
    const int32_t* tlen = spick3(S.tlen, slot);
    const int L = S.L;
    const int rt = (S.sb + 15) / 16, lt = (L + 15) / 16;
    const int li = lane & 15, lg = lane >> 4;
    const int nhc = (S.H + 15) / 16;
    __syncthreads();   // `red` may still be in use by the previous phase
    for (int item = blockIdx.x; item < rt * lt; item += gridDim.x) {
        const int t0 = (item / lt) * 16, l0 = (item % lt) * 16;
        v4f acc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = v4f{0.f, 0.f, 0.f, 0.f};
        {
            const int jl = l0 + li;
            const bool lok = jl < L;
            const int jlc = min(jl, L - 1);
            // A[i][k] = Yh[t0+i][hc0+k] (lane: i = li, k = lg); B[k][j] = x[head_col[hc0+k]][l0+j]
            const float* arow = Yh + (int64_t)(t0 + li) * S.Hp;   // padded rows are zero
            for (int c0 = wave; c0 < nhc; c0 += 4 * kNW) {
                float a[4][4], bv[4][4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int cc = min(c0 + u * kNW, nhc - 1);
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int hc = cc * 16 + 4 * k + lg;
                        a[u][k] = arow[hc];
                        bv[u][k] = S.x[(int64_t)S.head_col[min(hc, S.H - 1)] * L + jlc];
                    }
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (c0 + u * kNW < nhc) {
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const int hc = (c0 + u * kNW) * 16 + 4 * k + lg;
                            const float w = (hc < S.H && lok) ? bv[u][k] : 0.f;
                            acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][k], w, acc[k], 0, 0, 0);
                        }
                    }
                }
            }
        }
        const v4f g = acc[0] + acc[1] + acc[2] + acc[3];
#pragma unroll
        for (int v = 0; v < 4; ++v) red[(wave * 64 + lane) * 4 + v] = g[v];
        __syncthreads();
        {
            const int i = threadIdx.x >> 4, j = threadIdx.x & 15;   // 256 threads: 16 x 16
            const int t = t0 + i, jl = l0 + j;
            if (t < S.sb && jl < L) {
                const int q = 16 * (i >> 2) + j, v = i & 3;
                float r = red[q * 4 + v];
#pragma unroll
                for (int w = 1; w < kNW; ++w) r += red[(w * 64 + q) * 4 + v];
                const int nt = tlen[t];
                const int64_t base = (int64_t)t * S.maxlen;
                for (int k0 = 0; k0 < nt; k0 += 8) {
                    int cl[8];
                    float vl[8], xv[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int kk = min(k0 + u, nt - 1);
                        cl[u] = tcol[base + kk];
                        vl[u] = tval[base + kk];
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) xv[u] = S.x[(int64_t)cl[u] * L + jl];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        if (k0 + u < nt) r = fmaf(vl[u], xv[u], r);
                }
                S.r[(int64_t)t * L + jl] = r;
            }
        }
        __syncthreads();
    }
}

// Update of outer h for all lanes: x <- beta^s x + alpha * Y^T c.
//  * head columns: one workgroup per (16 head columns, 16 lanes) tile
//    computes Yh^T c (H x rows times rows x lanes) with FP32 MFMA 16x16x4;
//  * tail columns present in the block: one wave (or half-wave) per column
//    sums its bucket in increasing t for every lane (see below);
//  * all other columns: x <- beta^s x.
__device__ __forceinline__ void sparse_update(const Sparse& S, uint64_t h, int wave_id, int nwaves,
                                              int gtid, int nthreads, int64_t snap_row,
                                              int2* sorted, float* red) {
    const int lane = threadIdx.x & 63;
    const int slot = slot_of(h);
    const float* Yh = spick3(S.Yh, slot);
    const unsigned* bcnt = spick2(S.bcnt, (int)(h & 1));
    const int2* bent = spick2(S.bent, (int)(h & 1));
    const int L = S.L;
    const float alpha = (float)S.alpha_d;
    const int li = lane & 15, lg = lane >> 4;
    // Head columns: D[i][j] = sum_t Yh[t][hc0+i] c[t][l0+j]. One workgroup
    // per (16 head columns, 16 lanes) tile; wave w takes the 16-row chunks
    // w, w + 4, ... (four chunks of loads in flight) and the four partial
    // tiles are added in wave order through LDS (`red`, 4 KB).
    const int ht = (S.H + 15) / 16, lt = (L + 15) / 16;
    const int wave = wave_id % kNW;
    const int nch = (S.sb + 15) / 16;
    for (int item = blockIdx.x; item < ht * lt; item += gridDim.x) {
        const int hc0 = (item / lt) * 16, l0 = (item % lt) * 16;
        const int jl = l0 + li;
        const bool lok = jl < L;
        const int jlc = min(jl, L - 1);
        v4f acc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] = v4f{0.f, 0.f, 0.f, 0.f};
        for (int c0 = wave; c0 < nch; c0 += 4 * kNW) {
            float a[4][4], bv[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int ch = min(c0 + u * kNW, nch - 1);
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int t = ch * 16 + 4 * k + lg;   // < sbpad: padded rows are zero
                    a[u][k] = Yh[(int64_t)t * S.Hp + hc0 + li];
                    bv[u][k] = S.c[(int64_t)min(t, S.sb - 1) * L + jlc];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int ch = c0 + u * kNW;
                if (ch < nch) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const int t = ch * 16 + 4 * k + lg;
                        const float w = (t < S.sb && lok) ? bv[u][k] : 0.f;
                        acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[u][k], w, acc[k], 0, 0, 0);
                    }
                }
            }
        }
        const v4f g = acc[0] + acc[1] + acc[2] + acc[3];
#pragma unroll
        for (int v = 0; v < 4; ++v) red[(wave * 64 + lane) * 4 + v] = g[v];
        __syncthreads();
        if (wave == 0 && lok) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float d = red[lane * 4 + v];
#pragma unroll
                for (int w = 1; w < kNW; ++w) d += red[(w * 64 + lane) * 4 + v];
                const int hc = hc0 + 4 * lg + v;
                if (hc >= S.H) continue;
                const int64_t k = S.head_col[hc];
                const float xn = S.lbs[jl] * S.x[k * L + jl] + alpha * d;
                S.x[k * L + jl] = xn;
                if (!isfinite(xn)) raise_flag(S.flags, FLAG_NONFINITE);
                if (snap_row >= 0) S.x_hist[(snap_row * S.n + k) * L + jl] = xn;
            }
        }
        __syncthreads();
    }
    // Tail columns of the block, from the tail list: with at most 32 lanes
    // (and room for two scratch lists) each half-wave takes a column, else the
    // whole wave. Lane q of the group ranks bucket entries q and q + width by
    // (t, bucket slot) and stores them at their ranks in the group's LDS
    // scratch, then lane l (one per lambda lane) adds the entries in
    // increasing t, four loads in flight at a time.
    const int ncol = min((int)S.tlcnt[h & 1], (int)S.n);
    const int32_t* tl = spick2(S.tlist, (int)(h & 1));
    const int cpw = (L <= 32 && S.Hp >= 256) ? 2 : 1;   // columns per wave
    const int wd = kWave / cpw;                          // lanes per column
    const int half = lane / wd, hl = lane - half * wd;
    int2* srt = sorted + half * kBucketCap;
    // when the head tiles occupy only some workgroups, the others' waves take
    // the tail columns (the head tile costs about as much as their share)
    const int hw = ht * lt < (int)gridDim.x ? ht * lt * kNW : 0;   // waves with a head tile
    const int trank = wave_id - hw, ntw = nwaves - hw;
    for (int c0 = trank * cpw; trank >= 0 && c0 < ncol; c0 += ntw * cpw) {
        const int ci = c0 + half;
        const int ccol = tl[min(ci, ncol - 1)];
        const int cnt = ci < ncol ? min((int)bcnt[ccol], kBucketCap) : 0;
        const int2* be = bent + (int64_t)ccol * kBucketCap;
        const int2 none = make_int2(0x7fffffff, 0);
        const int2 e0 = hl < cnt ? be[hl] : none;
        const int2 e1 = hl + wd < cnt ? be[hl + wd] : none;
        int r0 = 0, r1 = 0;
        for (int q = 0; q < cnt; ++q) {
            const int tq = __shfl(q < wd ? e0.x : e1.x, q & (wd - 1), wd);
            r0 += (tq < e0.x || (tq == e0.x && q < hl)) ? 1 : 0;
            r1 += (tq < e1.x || (tq == e1.x && q < hl + wd)) ? 1 : 0;
        }
        wave_lds_sync();
        if (hl < cnt) srt[r0] = e0;
        if (hl + wd < cnt) srt[r1] = e1;
        wave_lds_sync();
        const int l = hl;
        if (ci < ncol && l < L) {
            float g = 0.f;
            int p = 0;
            for (; p + 4 <= cnt; p += 4) {
                const int2 e0v = srt[p], e1v = srt[p + 1], e2v = srt[p + 2], e3v = srt[p + 3];
                const float c0v = S.c[(int64_t)e0v.x * L + l], c1v = S.c[(int64_t)e1v.x * L + l],
                            c2v = S.c[(int64_t)e2v.x * L + l], c3v = S.c[(int64_t)e3v.x * L + l];
                g = fmaf(__int_as_float(e0v.y), c0v, g);
                g = fmaf(__int_as_float(e1v.y), c1v, g);
                g = fmaf(__int_as_float(e2v.y), c2v, g);
                g = fmaf(__int_as_float(e3v.y), c3v, g);
            }
            for (; p < cnt; ++p) {
                const int2 ev = srt[p];
                g = fmaf(__int_as_float(ev.y), S.c[(int64_t)ev.x * L + l], g);
            }
            const float xn = S.lbs[l] * S.x[(int64_t)ccol * L + l] + alpha * g;
            S.x[(int64_t)ccol * L + l] = xn;
            if (!isfinite(xn)) raise_flag(S.flags, FLAG_NONFINITE);
            if (snap_row >= 0) S.x_hist[(snap_row * S.n + ccol) * L + l] = xn;
        }
    }
    // Untouched columns: decay only. With L a multiple of 4 and 16-byte
    // aligned x (and history), four lanes at a time, four column pieces of
    // loads in flight per thread.
    const bool vec = (L & 3) == 0 && ((uintptr_t)S.x & 15) == 0 &&
                     (snap_row < 0 || ((uintptr_t)S.x_hist & 15) == 0);
    if (vec) {
        const int LQ = L >> 2;
        const int64_t nq = S.n * LQ;
        float4* x4 = reinterpret_cast<float4*>(S.x);
        const float4* lb4 = reinterpret_cast<const float4*>(S.lbs);
        for (int64_t base = gtid; base < nq; base += 4 * (int64_t)nthreads) {
            int hid[4];
            unsigned bc[4];
            float4 xv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t q = min(base + u * (int64_t)nthreads, nq - 1);
                const int64_t k = q / LQ;
                hid[u] = S.head_id[k];
                bc[u] = bcnt[k];
                xv[u] = x4[q];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t q = base + u * (int64_t)nthreads;
                if (q < nq && hid[u] < 0 && bc[u] == 0u) {
                    const float4 be = lb4[q % LQ];
                    const float4 xn = make_float4(be.x * xv[u].x, be.y * xv[u].y, be.z * xv[u].z,
                                                  be.w * xv[u].w);
                    x4[q] = xn;
                    if (snap_row >= 0) reinterpret_cast<float4*>(S.x_hist + snap_row * S.n * L)[q] = xn;
                }
            }
        }
        return;
    }
    for (int64_t q = gtid; q < S.n * L; q += nthreads) {
        const int64_t k = q / L;
        const int l = (int)(q - k * L);
        if (S.head_id[k] >= 0 || bcnt[k] != 0u) continue;
        const float xn = S.lbs[l] * S.x[q];
        S.x[q] = xn;
        if (snap_row >= 0) S.x_hist[snap_row * S.n * L + q] = xn;
    }
}

// Clear the bucket counts of outer h (every tail entry clears its column) and
// its tail list.
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
    if (gtid == 0) S.tlcnt[h & 1] = 0u;
}

// Rows of a recurrence pass and 16-byte prefix pieces per thread and batch.
constexpr int kRecRows = 8;
constexpr int kRecPieces = 2;

// Value of the lane whose index differs in bit 0 (CTRL 0xB1) or bit 1 (CTRL
// 0x4E) within each group of four lanes (DPP quad permutation).
template <int CTRL>
__device__ __forceinline__ float quad_perm(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double quad_perm(double v) {
    const long long x = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)x, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(x >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Residual corrections for lanes [l0, l0 + nl), nl <= kLanesPerRecWG, by the
// K workgroups of one lane group; workgroup k of the group owns rows
// [k b/K, (k+1) b/K) of every row block. In step j each takes its rows in
// passes of kRecRows: every thread covers all rows of the pass for its own
// 16-byte pieces of the row prefix (so each delta it reads from LDS serves
// all the rows), the per-thread sums are added in a fixed order through LDS
// (`red`), and one thread per (row, lane) forms z_j and delta_j. The deltas
// are published as tagged words and those of the other rows collected before
// step j + 1; the first batch of G pieces, the margins and the labels of the
// next step are loaded while waiting. The owner of a word clears it after the
// grid barrier that follows the recurrence, so every outer iteration starts
// from cleared words.
// LDS: dl (kLanesPerRecWG x sb ACC, lane-major), pw (kLanesPerRecWG x (s+1)
// ACC), red (kRecRows x kLanesPerRecWG x NT / 4 ACC).
template <typename ACC, int NT>
__device__ __forceinline__ void sparse_recurrence(const Sparse& S, const float* G, uint64_t h,
                                                  int l0, int nl, int k, int K, ACC* dl, ACC* pw,
                                                  ACC* red, unsigned long long spin) {
    constexpr int NL = kLanesPerRecWG;
    constexpr int RC = kRecRows, PB = kRecPieces;
    static_assert(RC * NL * 8 == NT, "one finishing group of 8 threads per (row, lane)");
    const int tid = threadIdx.x;
    const int b = S.b, s = S.s, sb = S.sb, L = S.L;
    const int RB = b / K, q_lo = k * RB;
    if (tid < NL) {
        ACC p = 1;
        const ACC be = tid < nl ? (ACC)S.lbeta[l0 + tid] : (ACC)1;
        for (int q = 0; q <= s; ++q) { pw[tid * (s + 1) + q] = p; p *= be; }
    }
    __syncthreads();
    const ACC alpha = (ACC)S.alpha_d;
    const float* yI = spick3(S.yI, slot_of(h));
    // finishing thread of (row o / NL, lane o % NL) of a pass: part == 0
    const int o = tid >> 3, part = tid & 7;
    const int orow = o / NL, olane = o - orow * NL;
    // First batch of G pieces of a step's first pass, and the finishing
    // threads' margins and labels, loaded one step ahead.
    float4 gp[RC][PB];
    float rp = 0.f, yp = 0.f;
    auto load_first = [&](int jj) {
        const int nvj = max((jj * b) >> 2, 1);
#pragma unroll
        for (int rr = 0; rr < RC; ++rr) {
            const int t = jj * b + q_lo + min(rr, RB - 1);
            const float4* g4 = reinterpret_cast<const float4*>(G + (int64_t)t * sb);
#pragma unroll
            for (int pb = 0; pb < PB; ++pb) gp[rr][pb] = g4[min(tid + pb * NT, nvj - 1)];
        }
        const int t = jj * b + q_lo + min(orow, RB - 1);
        rp = S.r[(int64_t)t * L + l0 + min(olane, nl - 1)];
        yp = yI[t];
    };
    load_first(0);
    for (int j = 0; j < s; ++j) {
        const int nv = (j * b) >> 2;   // 16-byte pieces of the row prefix
        for (int q0 = 0; q0 < RB; q0 += RC) {
            ACC acc[RC][NL];
#pragma unroll
            for (int rr = 0; rr < RC; ++rr)
#pragma unroll
                for (int l = 0; l < NL; ++l) acc[rr][l] = 0;
            for (int v0 = tid; v0 < nv; v0 += PB * NT) {
                float4 g[RC][PB];
                if (q0 == 0 && v0 == tid) {
#pragma unroll
                    for (int rr = 0; rr < RC; ++rr)
#pragma unroll
                        for (int pb = 0; pb < PB; ++pb) g[rr][pb] = gp[rr][pb];
                } else {
#pragma unroll
                    for (int rr = 0; rr < RC; ++rr) {
                        const int t = j * b + q_lo + min(q0 + rr, RB - 1);
                        const float4* g4 = reinterpret_cast<const float4*>(G + (int64_t)t * sb);
#pragma unroll
                        for (int pb = 0; pb < PB; ++pb) g[rr][pb] = g4[min(v0 + pb * NT, nv - 1)];
                    }
                }
#pragma unroll
                for (int pb = 0; pb < PB; ++pb) {
                    const int v = v0 + pb * NT;
                    const int e = 4 * min(v, nv - 1);
                    const int i = e / b;
                    ACC dv[NL][4], wl[NL];
#pragma unroll
                    for (int l = 0; l < NL; ++l) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) dv[l][q] = dl[l * sb + e + q];
                        wl[l] = v < nv ? pw[l * (s + 1) + (j - 1 - i)] : (ACC)0;
                    }
#pragma unroll
                    for (int rr = 0; rr < RC; ++rr)
#pragma unroll
                        for (int l = 0; l < NL; ++l) {
                            const ACC pt = (ACC)g[rr][pb].x * dv[l][0] + (ACC)g[rr][pb].y * dv[l][1] +
                                           (ACC)g[rr][pb].z * dv[l][2] + (ACC)g[rr][pb].w * dv[l][3];
                            acc[rr][l] += wl[l] * pt;
                        }
                }
            }
            // fixed-order sum over the threads: groups of four lanes first
            // (DPP), then thread (o, part) adds eight consecutive group sums
            // of output o, then the eight parts
            constexpr int NG = NT / 4;
#pragma unroll
            for (int rr = 0; rr < RC; ++rr)
#pragma unroll
                for (int l = 0; l < NL; ++l) {
                    ACC a = acc[rr][l];
                    a += quad_perm<0xB1>(a);
                    a += quad_perm<0x4E>(a);
                    if ((tid & 3) == 0) red[(rr * NL + l) * NG + (tid >> 2)] = a;
                }
            __syncthreads();
            ACC tot = 0;
#pragma unroll
            for (int m = 0; m < NG / 8; ++m) tot += red[o * NG + part * (NG / 8) + m];
            tot += shfl_xor(tot, 1);
            tot += shfl_xor(tot, 2);
            tot += shfl_xor(tot, 4);
            const int q = q0 + orow;
            if (part == 0 && q < RB) {
                const int t = j * b + q_lo + q;
                const int l = olane;
                float rv = rp, yv = yp;
                if (q0 != 0) {
                    rv = S.r[(int64_t)t * L + l0 + min(l, nl - 1)];
                    yv = yI[t];
                }
                ACC d = 0;
                if (l < nl) {
                    const ACC z = pw[l * (s + 1) + j] * (ACC)rv + alpha * tot;
                    d = glm_delta<ACC>(z, (ACC)yv, S.loss);
                    if (!isfinite(z) || !isfinite(d)) raise_flag(S.flags, FLAG_NONFINITE);
                    S.c[(int64_t)t * L + l0 + l] = (float)(pw[l * (s + 1) + (s - 1 - j)] * d);
                    if (K > 1 && j + 1 < s) pub_put(S.pub + 2 * ((int64_t)t * L + l0 + l), d);
                }
                dl[l * sb + t] = d;
            }
            __syncthreads();   // `red` is reused by the next pass
        }
        if (j + 1 < s) load_first(j + 1);
        if (K > 1 && j + 1 < s) {
            // Deltas of the rows the other workgroups of the group own, four
            // per thread at a time: all their words are read, then the ones
            // still missing are read again.
            constexpr int kP = 4;
            for (int w0 = tid; w0 < b * NL; w0 += kP * NT) {
                const unsigned long long* pp[kP];
                ACC d[kP];
                bool need[kP];
#pragma unroll
                for (int u = 0; u < kP; ++u) {
                    const int w = w0 + u * NT;
                    const int qq = w / NL, l = w - qq * NL;
                    need[u] = w < b * NL && (qq < q_lo || qq >= q_lo + RB) && l < nl;
                    pp[u] = S.pub + 2 * ((int64_t)(j * b + min(qq, b - 1)) * L + l0 + min(l, nl - 1));
                    d[u] = 0;
                }
                unsigned long long n = 0;
                for (;;) {
                    bool all = true;
#pragma unroll
                    for (int u = 0; u < kP; ++u)
                        if (need[u]) {
                            need[u] = !pub_get(pp[u], d[u]);
                            all = all && !need[u];
                        }
                    if (all) break;
                    if (++n > spin) {
                        raise_flag(S.flags, FLAG_TIMEOUT);
                        break;
                    }
                    if ((n & 63ull) == 0 && atomic_load_relaxed(S.flags + FLAG_TIMEOUT)) break;
                    __builtin_amdgcn_s_sleep(1);
                }
#pragma unroll
                for (int u = 0; u < kP; ++u) {
                    const int w = w0 + u * NT;
                    const int qq = w / NL;
                    if (w < b * NL && (qq < q_lo || qq >= q_lo + RB))
                        dl[(w - qq * NL) * sb + j * b + qq] = d[u];
                }
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

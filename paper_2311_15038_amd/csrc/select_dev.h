// Device-side pieces of threshold selection shared by the single-volume
// launches and the batched persistent kernel: block primitives over one
// 1024-thread workgroup, the smoothed-histogram chunk, the stages (per-chunk
// pass, per-chunk search, finish) and one row of the keep mask.
#pragma once

#include "common.h"

namespace vr {
namespace sel {

constexpr int kT = 1024;                  // threads = bins per chunk
constexpr int kB = VR_NBINS;
constexpr int kMaxChunks = kB / kT;       // 64
constexpr int kMaxRadius = kT - 1;
constexpr int kHalo = kT + 2 * kMaxRadius + 2;   // smoothed-sum window of a chunk

struct ValleyChunk {      // launch 1 (valley)
    uint64_t smax;
    uint32_t arg;
    uint32_t pad;
};
struct ValleyCand {       // launch 2 (valley)
    int32_t cand;         // first qualifying bin, or kB
    int32_t chg_below;    // last change point below cand (>= p), or -1
    int32_t chg_all;      // last change point in the chunk (>= p), or -1
    int32_t pad;
};
struct SumChunk {         // launch 1 (Otsu, ITS)
    uint64_t n, s;
};
struct OtsuChunk {        // launch 2 (Otsu)
    double sigma;
    int32_t T;
    int32_t pad;
};
struct ItsChunk {         // launch 1 extra (ITS): occupied range of the chunk
    int32_t lo, hi;
};
// layout of the 8 KiB scratch: [0, 1024) launch-1 records, [1024, 2048) launch-2 records,
// [2048, 2560) ITS ranges
static_assert(sizeof(ValleyChunk) * kMaxChunks <= 1024, "scratch");
static_assert(sizeof(SumChunk) * kMaxChunks <= 1024, "scratch");
static_assert(sizeof(ValleyCand) * kMaxChunks <= 1024, "scratch");
static_assert(sizeof(OtsuChunk) * kMaxChunks <= 1024, "scratch");

// LDS of a selection workgroup (shared by the three stages).
struct SelLds {
    uint64_t X[kHalo];
    uint64_t cb[kT];          // coarse bins of a chunk (Otsu, ITS with bin width > 1)
    uint64_t wsum[kT / 64];
    uint64_t kbuf[kT];
    int ibuf[kT];
    double dbuf[kT];
    SumChunk sums[kMaxChunks];
    uint32_t s_res[4];
    int s_T, s_done, s_it;
};

__device__ __forceinline__ uint64_t hv(const uint64_t* H, int b) { return (b >= 0 && b < kB) ? H[b] : 0; }

// sum of the 2^k (k >= 1) fine bins from f (even), in 16-byte loads issued together
template <int N>
__device__ __forceinline__ uint64_t sum_run(const uint64_t* __restrict__ H, int64_t f)
{
    const uint4* p = reinterpret_cast<const uint4*>(H + f);
    uint4 q[N];
#pragma unroll
    for (int i = 0; i < N; ++i) q[i] = p[i];
    uint64_t s = 0;
#pragma unroll
    for (int i = 0; i < N; ++i) s += ((uint64_t)q[i].y << 32 | q[i].x) + ((uint64_t)q[i].w << 32 | q[i].z);
    return s;
}

__device__ __forceinline__ uint64_t sum_fine(const uint64_t* __restrict__ H, int64_t f, int n)
{
    switch (n) {
    case 2: return sum_run<1>(H, f);
    case 4: return sum_run<2>(H, f);
    case 8: return sum_run<4>(H, f);
    case 16: return sum_run<8>(H, f);
    case 32: return sum_run<16>(H, f);
    default: return sum_run<32>(H, f);   // 64
    }
}

// Coarse bin c * kT + t (width 2^shift, 0 past the last one) for thread t of
// the workgroup.  Up to 32 fine bins per coarse bin, each thread sums its own;
// from 64 up, each thread sums a run of 64 fine bins and adds it to its coarse
// bin in LDS (cb) with one atomic, and with `fresh` false the sums of the
// previous call on the same chunk are reused.  Every thread must call it.
__device__ inline uint64_t chunk_coarse(const uint64_t* __restrict__ H, int c, int shift, uint64_t* cb,
                                        bool fresh = true)
{
    const int t = threadIdx.x, b = c * kT + t;
    if (shift == 0) return hv(H, b);
    const int nb = kB >> shift;
    if (shift < 6) return b < nb ? sum_fine(H, (int64_t)b << shift, 1 << shift) : 0;
    if (fresh) {
        cb[t] = 0;
        __syncthreads();
        const int64_t f0 = ((int64_t)c * kT) << shift;
        const int64_t f = f0 + (int64_t)t * 64;
        if (f < kB) {
            const uint64_t v = sum_fine(H, f, 64);
            if (v) atomicAdd(reinterpret_cast<unsigned long long*>(cb + ((f >> shift) - (int64_t)c * kT)),
                             (unsigned long long)v);
        }
        __syncthreads();
    }
    return b < nb ? cb[t] : 0;
}

// ------------------------------------------------------------ block primitives
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint64_t x = __shfl_up(v, off);
        if (lane >= off) v += x;
    }
    return v;
}

// Inclusive scan of one value per thread over the block; returns the block total too.
__device__ inline uint64_t block_incl_scan(uint64_t v, uint64_t* wsum, uint64_t& total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_incl_scan(v);
    if (lane == 63) wsum[w] = v;
    __syncthreads();
    if (w == 0) {
        uint64_t x = lane < kT / 64 ? wsum[lane] : 0;
        x = wave_incl_scan(x);
        if (lane < kT / 64) wsum[lane] = x;
    }
    __syncthreads();
    const uint64_t base = w > 0 ? wsum[w - 1] : 0;
    total = wsum[kT / 64 - 1];
    __syncthreads();
    return v + base;
}

// (key, index): larger key wins, ties -> smaller index.
template <typename K>
__device__ inline void block_argmax(K key, int idx, K* kbuf, int* ibuf, K& okey, int& oidx)
{
    const int t = threadIdx.x;
    kbuf[t] = key;
    ibuf[t] = idx;
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if (t < s) {
            const K a = kbuf[t], b = kbuf[t + s];
            const int ia = ibuf[t], ib = ibuf[t + s];
            if (b > a || (b == a && ib < ia)) {
                kbuf[t] = b;
                ibuf[t] = ib;
            }
        }
        __syncthreads();
    }
    okey = kbuf[0];
    oidx = ibuf[0];
    __syncthreads();
}

__device__ inline int block_min_i(int v, int* buf)
{
    const int t = threadIdx.x;
    buf[t] = v;
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if (t < s && buf[t + s] < buf[t]) buf[t] = buf[t + s];
        __syncthreads();
    }
    const int r = buf[0];
    __syncthreads();
    return r;
}

__device__ inline int block_max_i(int v, int* buf) { return -block_min_i(-v, buf); }

// Smoothed histogram of this chunk: S[b] for b = base + t and S[b + 1].
// X holds H over [base - r - 1, base + kT + r] (zero outside [0, B)) and is
// turned into its inclusive prefix, so S[b] = X[b + r] - X[b - r - 1].
__device__ inline void chunk_smoothed(const uint64_t* H, int base, int r, uint64_t* X, uint64_t* wsum,
                               uint64_t& S0, uint64_t& S1)
{
    const int lo = base - r - 1;
    const int m = kT + 2 * r + 2;
    const int per = (m + kT - 1) / kT;       // <= 3 consecutive values per thread
    const int t = threadIdx.x;
    for (int i = t; i < m; i += kT) X[i] = hv(H, lo + i);
    __syncthreads();
    uint64_t run = 0;
    for (int j = 0; j < per; ++j) {
        const int i = t * per + j;
        if (i < m) run += X[i];
    }
    uint64_t total;
    const uint64_t incl = block_incl_scan(run, wsum, total);
    uint64_t acc = incl - run;
    for (int j = 0; j < per; ++j) {
        const int i = t * per + j;
        if (i < m) {
            acc += X[i];
            X[i] = acc;
        }
    }
    __syncthreads();
    const int b = base + t;
    // S[b] = Q[b + r] - Q[b - r - 1], indices relative to lo
    S0 = X[b + r - lo] - X[b - r - 1 - lo];
    S1 = X[b + 1 + r - lo] - X[b - r - lo];
}

// ------------------------------------------------------------ launch 1
__device__ inline void chunk_pass(SelLds& Ls, int c, const uint64_t* __restrict__ H, int rule, int param,
                                  uint32_t* __restrict__ scratch)
{
    uint64_t* X = Ls.X;
    uint64_t* wsum = Ls.wsum;
    uint64_t* kbuf = Ls.kbuf;
    int* ibuf = Ls.ibuf;
    const int t = threadIdx.x, base = c * kT;
    if (rule == VR_RULE_VALLEY) {
        uint64_t S0, S1;
        chunk_smoothed(H, base, param, X, wsum, S0, S1);
        uint64_t m;
        int a;
        block_argmax<uint64_t>(S0, base + t, kbuf, ibuf, m, a);
        if (t == 0) {
            auto* rec = reinterpret_cast<ValleyChunk*>(scratch) + c;
            rec->smax = m;
            rec->arg = (uint32_t)a;
        }
    } else {
        const int b = base + t;
        const uint64_t h = chunk_coarse(H, c, param, Ls.cb);
        uint64_t tn, ts;
        block_incl_scan(h, wsum, tn);
        block_incl_scan((uint64_t)b * h, wsum, ts);
        const int lo = block_min_i(h ? b : kB, ibuf);
        const int hi = block_max_i(h ? b : -1, ibuf);
        if (t == 0) {
            auto* rec = reinterpret_cast<SumChunk*>(scratch) + c;
            rec->n = tn;
            rec->s = ts;
            auto* rng = reinterpret_cast<ItsChunk*>(reinterpret_cast<char*>(scratch) + 2048) + c;
            rng->lo = lo;
            rng->hi = hi;
        }
    }
}

// ------------------------------------------------------------ launch 2
__device__ inline void chunk_search(SelLds& Ls, int c, const uint64_t* __restrict__ H, int rule, int param,
                                    int n_chunks, uint32_t* __restrict__ scratch)
{
    uint64_t* X = Ls.X;
    uint64_t* wsum = Ls.wsum;
    uint64_t* kbuf = Ls.kbuf;
    int* ibuf = Ls.ibuf;
    double* dbuf = Ls.dbuf;
    const int t = threadIdx.x, base = c * kT;
    char* sc = reinterpret_cast<char*>(scratch);
    if (rule == VR_RULE_VALLEY) {
        // global peak p = first argmax over the chunk records
        const auto* rec = reinterpret_cast<const ValleyChunk*>(sc);
        uint64_t Sp;
        int p;
        block_argmax<uint64_t>(t < n_chunks ? rec[t].smax : 0, t < n_chunks ? (int)rec[t].arg : kB,
                               kbuf, ibuf, Sp, p);
        uint64_t S0, S1;
        chunk_smoothed(H, base, param, X, wsum, S0, S1);
        const int b = base + t;
        const bool inr = b <= kB - 2;             // S[b + 1] exists
        const bool qual = inr && b > p && 2 * S0 <= Sp && S1 > S0;
        const bool chg = inr && b >= p && S1 != S0;
        const int cand = block_min_i(qual ? b : kB, ibuf);
        const int below = block_max_i(chg && b < cand ? b : -1, ibuf);
        const int all = block_max_i(chg ? b : -1, ibuf);
        if (t == 0) {
            auto* out = reinterpret_cast<ValleyCand*>(sc + 1024) + c;
            out->cand = cand;
            out->chg_below = below;
            out->chg_all = all;
        }
    } else {
        // Otsu: T = b; class a = coarse bins [0, T), class b = [T, B-1]
        const auto* rec = reinterpret_cast<const SumChunk*>(sc);
        uint64_t n0 = 0, s0 = 0, N = 0, Stot = 0;
        for (int k = 0; k < n_chunks; ++k) {
            N += rec[k].n;
            Stot += rec[k].s;
            if (k < c) {
                n0 += rec[k].n;
                s0 += rec[k].s;
            }
        }
        const int B = kB >> param;
        const int T = base + t;
        const uint64_t h = chunk_coarse(H, c, param, Ls.cb);
        uint64_t tn, ts;
        const uint64_t in_n = block_incl_scan(h, wsum, tn);
        const uint64_t in_s = block_incl_scan((uint64_t)T * h, wsum, ts);
        const uint64_t na = n0 + in_n - h, sa = s0 + in_s - (uint64_t)T * h;   // exclusive at T
        double sigma = 0.0;
        const uint64_t nb = N - na;
        if (T < B && na != 0 && nb != 0) {
            const uint64_t sb = Stot - sa;
            const double w_a = __ddiv_rn((double)na, (double)N);
            const double w_b = __ddiv_rn((double)nb, (double)N);
            const double u_a = __ddiv_rn((double)sa, (double)na);
            const double u_b = __ddiv_rn((double)sb, (double)nb);
            const double d = __dsub_rn(u_a, u_b);
            sigma = __dmul_rn(__dmul_rn(w_a, w_b), __dmul_rn(d, d));
        }
        double best;
        int bT;
        block_argmax<double>(sigma, sigma > 0.0 ? T : kB, dbuf, ibuf, best, bT);
        if (t == 0) {
            auto* out = reinterpret_cast<OtsuChunk*>(sc + 1024) + c;
            out->sigma = best;
            out->T = bT;
        }
    }
}

// ------------------------------------------------------------ launch 3
// One 1024-bin row j of the keep mask: keep[b] = b >= T and no top-slice
// count at b; a wave's 64 consecutive bins become two words by ballot.
__device__ __forceinline__ void mask_row(const uint64_t* __restrict__ Htop, uint32_t T, int j,
                                         uint32_t* __restrict__ bits)
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const uint32_t b = (uint32_t)(j * kT + t);
    const uint64_t m = __ballot(b >= T && (Htop == nullptr || Htop[b] == 0));
    if (lane == 0) {
        bits[32 * j + 2 * w] = (uint32_t)m;
        bits[32 * j + 2 * w + 1] = (uint32_t)(m >> 32);
    }
}

// Combines the chunk records into the threshold and writes the result; with
// write_mask the same workgroup then writes the whole keep mask (otherwise a
// separate launch of mask_row workgroups does, after this one).
__device__ inline void finish(SelLds& Ls, const uint64_t* __restrict__ H, const uint64_t* __restrict__ Htop,
                              int rule, int param, int n_chunks, uint32_t* __restrict__ result,
                              uint32_t* __restrict__ bits, bool write_mask = true)
{
    uint64_t* wsum = Ls.wsum;
    int* ibuf = Ls.ibuf;
    uint64_t* kbuf = Ls.kbuf;
    double* dbuf = Ls.dbuf;
    uint32_t* s_res = Ls.s_res;
    int& s_T = Ls.s_T;
    int& s_done = Ls.s_done;
    int& s_it = Ls.s_it;
    SumChunk* sums = Ls.sums;
    const int t = threadIdx.x;
    const char* sc = reinterpret_cast<const char*>(bits);
    if (rule == VR_RULE_VALLEY) {
        const auto* rec = reinterpret_cast<const ValleyChunk*>(sc);
        const auto* cnd = reinterpret_cast<const ValleyCand*>(sc + 1024);
        uint64_t Sp;
        int p;
        block_argmax<uint64_t>(t < n_chunks ? rec[t].smax : 0, t < n_chunks ? (int)rec[t].arg : kB,
                               kbuf, ibuf, Sp, p);
        const int bstar = block_min_i(t < n_chunks ? cnd[t].cand : kB, ibuf);
        if (bstar >= kB) {
            if (t == 0) { s_res[0] = kB - 1; s_res[1] = (uint32_t)p; s_res[2] = 0xFFFFFFFFu; s_res[3] = 0; }
        } else {
            const int cs = bstar / kT;
            int v = -1;
            if (t < cs) v = cnd[t].chg_all;
            else if (t == cs) v = cnd[t].chg_below;
            const int last = block_max_i(v, ibuf);
            if (t == 0) { s_res[0] = (uint32_t)(last + 1); s_res[1] = (uint32_t)p; s_res[2] = (uint32_t)bstar; s_res[3] = 0; }
        }
    } else if (rule == VR_RULE_OTSU) {
        const auto* oc = reinterpret_cast<const OtsuChunk*>(sc + 1024);
        double best;
        int bT;
        block_argmax<double>(t < n_chunks ? oc[t].sigma : 0.0, t < n_chunks && oc[t].sigma > 0.0 ? oc[t].T : kB,
                             dbuf, ibuf, best, bT);
        if (t == 0) { s_res[0] = best > 0.0 ? (uint32_t)(bT << param) : 0u; s_res[1] = 0; s_res[2] = 0; s_res[3] = 0; }
    } else if (rule == VR_RULE_ITS) {
        // isodata from the middle of the occupied range, T <- floor((mu_1 + mu_2) * 0.5)
        const auto* rec = reinterpret_cast<const SumChunk*>(sc);
        const auto* rng = reinterpret_cast<const ItsChunk*>(sc + 2048);
        if (t < n_chunks) sums[t] = rec[t];
        const int bmin = block_min_i(t < n_chunks ? rng[t].lo : kB, ibuf);
        const int bmax = block_max_i(t < n_chunks ? rng[t].hi : -1, ibuf);
        uint64_t N = 0, Stot = 0;
        for (int k = 0; k < n_chunks; ++k) { N += sums[k].n; Stot += sums[k].s; }
        if (bmax < 0) {
            if (t == 0) { s_res[0] = 0; s_res[1] = 0; s_res[2] = 0; s_res[3] = 0; }
        } else {
            if (t == 0) { s_T = (bmin + bmax + 1) / 2; s_done = 0; s_it = 0; }
            __syncthreads();
            int c_prev = -1;
            for (int guard = 0; guard < 1000; ++guard) {
                const int T = s_T;
                // n_1, s_1 over coarse bins [0, T): whole chunks plus the part of chunk T / kT
                const int c = T / kT;
                const int b = c * kT + t;
                const uint64_t hb = chunk_coarse(H, c, param, Ls.cb, c != c_prev);
                c_prev = c;
                const uint64_t h = b < T ? hb : 0;
                uint64_t pn, ps;
                block_incl_scan(h, wsum, pn);
                block_incl_scan((uint64_t)b * h, wsum, ps);
                if (t == 0) {
                    uint64_t n1 = pn, s1 = ps;
                    for (int k = 0; k < c; ++k) { n1 += sums[k].n; s1 += sums[k].s; }
                    s_it += 1;
                    const uint64_t n2 = N - n1, s2 = Stot - s1;
                    if (n1 == 0 || n2 == 0) {
                        s_done = 1;
                    } else {
                        const double mu1 = __ddiv_rn((double)s1, (double)n1);
                        const double mu2 = __ddiv_rn((double)s2, (double)n2);
                        const int Tn = (int)floor(__dmul_rn(__dadd_rn(mu1, mu2), 0.5));
                        if (Tn == T) s_done = 1;
                        else s_T = Tn;
                    }
                }
                __syncthreads();
                if (s_done) break;
            }
            if (t == 0) { s_res[0] = (uint32_t)(s_T << param); s_res[1] = (uint32_t)s_it; s_res[2] = 0; s_res[3] = 0; }
        }
    } else {
        if (t == 0) { s_res[0] = 0; s_res[1] = 0; s_res[2] = 0; s_res[3] = 0; }
    }
    __syncthreads();          // every read of the scratch is done before the mask overwrites it
    const uint32_t T = s_res[0];
    if (t < 4) result[t] = s_res[t];
    if (write_mask)
        for (int j = 0; j < kB / kT; ++j) mask_row(Htop, T, j, bits);
}

}  // namespace sel
}  // namespace vr

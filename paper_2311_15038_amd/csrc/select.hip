// Threshold selection and keep mask on the device (Sections III-A and III-D).
//
// One workgroup of 1024 threads; thread t owns a contiguous run of bins.  The
// valley rule works on a box-smoothed copy of the 65536-bin histogram that is
// recomputed by sliding windows (never materialised); Otsu (Algorithm 1) and
// ITS (Algorithm 2) work on bins of width 2^shift, summed on the fly from the
// fine histogram.  Floating point that decides a threshold uses IEEE FP64
// operations written out one by one (no contraction), in the order given
// alongside each rule, so the integer result is reproducible on any IEEE FP64
// machine that evaluates the same expressions.
#include "common.h"

namespace {

constexpr int kT = 1024;
constexpr int kB = VR_NBINS;

struct Red {
    uint64_t u[kT];
    double d[kT];
    int i[kT];
};

// Block reduction of (key, index): larger key wins, ties -> smaller index.
// Returns the winner's (key, index) to every thread.
__device__ void reduce_max_u64(Red& r, uint64_t key, int idx, uint64_t& okey, int& oidx)
{
    const int t = threadIdx.x;
    __syncthreads();
    r.u[t] = key;
    r.i[t] = idx;
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if (t < s) {
            uint64_t a = r.u[t], b = r.u[t + s];
            int ia = r.i[t], ib = r.i[t + s];
            if (b > a || (b == a && ib < ia)) {
                r.u[t] = b;
                r.i[t] = ib;
            }
        }
        __syncthreads();
    }
    okey = r.u[0];
    oidx = r.i[0];
}

__device__ void reduce_max_f64(Red& r, double key, int idx, double& okey, int& oidx)
{
    const int t = threadIdx.x;
    __syncthreads();
    r.d[t] = key;
    r.i[t] = idx;
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if (t < s) {
            double a = r.d[t], b = r.d[t + s];
            int ia = r.i[t], ib = r.i[t + s];
            if (b > a || (b == a && ib < ia)) {
                r.d[t] = b;
                r.i[t] = ib;
            }
        }
        __syncthreads();
    }
    okey = r.d[0];
    oidx = r.i[0];
}

// min (or max with sign flip by the caller) of an int over the block
__device__ int reduce_min_i(Red& r, int v)
{
    const int t = threadIdx.x;
    __syncthreads();
    r.i[t] = v;
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if (t < s && r.i[t + s] < r.i[t]) r.i[t] = r.i[t + s];
        __syncthreads();
    }
    return r.i[0];
}

// Exclusive block scan of two u64 values; also returns the totals.
__device__ void scan2(Red& r, uint64_t a, uint64_t b, uint64_t& ea, uint64_t& eb, uint64_t& ta,
                      uint64_t& tb)
{
    __shared__ uint64_t sb[kT];
    const int t = threadIdx.x;
    __syncthreads();
    r.u[t] = a;
    sb[t] = b;
    __syncthreads();
    for (int off = 1; off < kT; off <<= 1) {
        uint64_t xa = t >= off ? r.u[t - off] : 0, xb = t >= off ? sb[t - off] : 0;
        __syncthreads();
        r.u[t] += xa;
        sb[t] += xb;
        __syncthreads();
    }
    ta = r.u[kT - 1];
    tb = sb[kT - 1];
    ea = r.u[t] - a;
    eb = sb[t] - b;
    __syncthreads();
}

__device__ __forceinline__ uint64_t hv(const uint64_t* H, int b) { return (b >= 0 && b < kB) ? H[b] : 0; }

__device__ uint64_t window(const uint64_t* H, int b, int r)
{
    uint64_t s = 0;
    for (int k = b - r; k <= b + r; ++k) s += hv(H, k);
    return s;
}

// ---------------------------------------------------------------- valley
// p = first argmax of S; b* = first b > p with 2 S[b] <= S[p] and S[b+1] > S[b];
// T = first bin of the plateau of S ending at b*; 65535 if there is no b*.
__device__ void valley(Red& red, const uint64_t* H, int r, uint32_t* out)
{
    __shared__ uint64_t s_bstar_val;
    const int t = threadIdx.x;
    const int per = kB / kT, b0 = t * per;

    uint64_t S = window(H, b0, r), best = S;
    int bi = b0;
    for (int j = 1; j < per; ++j) {
        const int b = b0 + j;
        S = S + hv(H, b + r) - hv(H, b - r - 1);
        if (S > best) { best = S, bi = b; }
    }
    uint64_t Sp;
    int p;
    reduce_max_u64(red, best, bi, Sp, p);

    // first b > p past half height where S rises
    int cand = kB;
    S = window(H, b0, r);
    for (int j = 0; j < per && b0 + j < kB - 1; ++j) {
        const int b = b0 + j;
        const uint64_t Sn = S + hv(H, b + 1 + r) - hv(H, b - r);
        if (b > p && 2 * S <= Sp && Sn > S && cand == kB) cand = b;
        S = Sn;
    }
    const int bstar = reduce_min_i(red, cand);
    if (bstar >= kB) {
        if (t == 0) { out[0] = kB - 1; out[1] = (uint32_t)p; out[2] = 0xFFFFFFFFu; out[3] = 0; }
        return;
    }
    if (t == 0) s_bstar_val = window(H, bstar, r);
    __syncthreads();
    const uint64_t Sb = s_bstar_val;
    // last b in [p, b*) with S[b] != S[b*]; T is the bin after it
    int last = -1;
    S = window(H, b0, r);
    for (int j = 0; j < per; ++j) {
        const int b = b0 + j;
        if (j > 0) S = S + hv(H, b + r) - hv(H, b - r - 1);
        if (b >= p && b < bstar && S != Sb) last = b;
    }
    const int neg = reduce_min_i(red, -last);
    if (t == 0) {
        out[0] = (uint32_t)(-neg + 1);
        out[1] = (uint32_t)p;
        out[2] = (uint32_t)bstar;
        out[3] = 0;
    }
}

// coarse bin b of width 2^shift
__device__ __forceinline__ uint64_t coarse(const uint64_t* H, int b, int shift)
{
    uint64_t s = 0;
    const int w = 1 << shift;
    for (int k = 0; k < w; ++k) s += H[(b << shift) + k];
    return s;
}

// ---------------------------------------------------------------- Otsu
// Algorithm 1: for T = 0..B-1, class a = [0, T), class b = [T, B-1]:
//   w_a = n_a / N, w_b = n_b / N, u_a = s_a / n_a, u_b = s_b / n_b,
//   sigma = (w_a * w_b) * ((u_a - u_b) * (u_a - u_b)); strictly greater wins.
__device__ void otsu(Red& red, const uint64_t* H, int shift, uint32_t* out)
{
    const int t = threadIdx.x;
    const int B = kB >> shift;
    const int per = (B + kT - 1) / kT;
    const int b0 = t * per;
    uint64_t n_loc = 0, s_loc = 0;
    for (int j = 0; j < per && b0 + j < B; ++j) {
        const uint64_t h = coarse(H, b0 + j, shift);
        n_loc += h;
        s_loc += (uint64_t)(b0 + j) * h;
    }
    uint64_t na, sa, N, Stot;
    scan2(red, n_loc, s_loc, na, sa, N, Stot);
    double best = 0.0;
    int bestT = 0;
    for (int j = 0; j < per && b0 + j < B; ++j) {
        const int T = b0 + j;
        // class a holds bins < T: n_a, s_a are the exclusive prefix at T
        const uint64_t nb = N - na;
        if (na != 0 && nb != 0) {
            const uint64_t sb = Stot - sa;
            const double w_a = __ddiv_rn((double)na, (double)N);
            const double w_b = __ddiv_rn((double)nb, (double)N);
            const double u_a = __ddiv_rn((double)sa, (double)na);
            const double u_b = __ddiv_rn((double)sb, (double)nb);
            const double d = __dsub_rn(u_a, u_b);
            const double sigma = __dmul_rn(__dmul_rn(w_a, w_b), __dmul_rn(d, d));
            if (sigma > best) { best = sigma; bestT = T; }
        }
        const uint64_t h = coarse(H, T, shift);
        na += h;
        sa += (uint64_t)T * h;
    }
    double bv;
    int bT;
    // a thread with no candidate reports (0, large index) so it never wins a tie
    reduce_max_f64(red, best, best > 0.0 ? bestT : kB, bv, bT);
    if (t == 0) {
        out[0] = bv > 0.0 ? (uint32_t)(bT << shift) : 0u;
        out[1] = 0;
        out[2] = 0;
        out[3] = 0;
    }
}

// ---------------------------------------------------------------- ITS
// Algorithm 2 as isodata: T starts at (b_min + b_max + 1) / 2 over non-empty
// bins; mu_1 = s_1 / n_1 over [0, T), mu_2 = s_2 / n_2 over [T, B-1];
// T <- floor((mu_1 + mu_2) * 0.5) until T repeats or a class is empty.
__device__ void its(Red& red, const uint64_t* H, int shift, uint32_t* out)
{
    __shared__ uint64_t s_n1, s_s1;
    __shared__ int s_T, s_done, s_it;
    const int t = threadIdx.x;
    const int B = kB >> shift;
    const int per = (B + kT - 1) / kT;
    const int b0 = t * per;
    uint64_t n_loc = 0, s_loc = 0;
    int lo = kB, hi = -1;
    for (int j = 0; j < per && b0 + j < B; ++j) {
        const uint64_t h = coarse(H, b0 + j, shift);
        n_loc += h;
        s_loc += (uint64_t)(b0 + j) * h;
        if (h) {
            if (b0 + j < lo) lo = b0 + j;
            hi = b0 + j;
        }
    }
    uint64_t nbase, sbase, N, Stot;
    scan2(red, n_loc, s_loc, nbase, sbase, N, Stot);
    const int bmin = reduce_min_i(red, lo);
    const int bmax = -reduce_min_i(red, -hi);
    if (bmax < 0) {
        if (t == 0) { out[0] = 0; out[1] = 0; out[2] = 0; out[3] = 0; }
        return;
    }
    if (t == 0) { s_T = (bmin + bmax + 1) / 2; s_done = 0; s_it = 0; }
    __syncthreads();
    for (int guard = 0; guard < 1000; ++guard) {
        const int T = s_T;
        // the owner of bin T supplies n_1, s_1 = sums over [0, T)
        if (T >= b0 && T < b0 + per && T < B) {
            uint64_t n1 = nbase, s1 = sbase;
            for (int b = b0; b < T; ++b) {
                const uint64_t h = coarse(H, b, shift);
                n1 += h;
                s1 += (uint64_t)b * h;
            }
            s_n1 = n1;
            s_s1 = s1;
        }
        if (t == 0 && T >= B) { s_n1 = N; s_s1 = Stot; }
        __syncthreads();
        if (t == 0) {
            s_it += 1;
            const uint64_t n1 = s_n1, s1 = s_s1, n2 = N - n1, s2 = Stot - s1;
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
    if (t == 0) {
        out[0] = (uint32_t)(s_T << shift);
        out[1] = (uint32_t)s_it;
        out[2] = 0;
        out[3] = 0;
    }
}

__global__ void __launch_bounds__(kT)
select_kernel(const uint64_t* __restrict__ H, const uint64_t* __restrict__ Htop, int rule, int param,
              uint32_t* __restrict__ out, uint32_t* __restrict__ bits)
{
    __shared__ Red red;
    __shared__ uint32_t s_T;
    if (rule == VR_RULE_VALLEY) valley(red, H, param, out);
    else if (rule == VR_RULE_OTSU) otsu(red, H, param, out);
    else if (rule == VR_RULE_ITS) its(red, H, param, out);
    else if (threadIdx.x == 0) { out[0] = 0; out[1] = 0; out[2] = 0; out[3] = 0; }
    __syncthreads();
    // every thread of this block wrote `out` through thread 0 only; make it visible
    __threadfence_block();
    if (threadIdx.x == 0) s_T = out[0];
    __syncthreads();
    const uint32_t T = s_T;
    for (int w = threadIdx.x; w < VR_KEEP_WORDS; w += kT) {
        uint32_t m = 0;
        for (int j = 0; j < 32; ++j) {
            const uint32_t b = (uint32_t)w * 32u + (uint32_t)j;
            const bool keep = b >= T && (Htop == nullptr || Htop[b] == 0);
            m |= (keep ? 1u : 0u) << j;
        }
        bits[w] = m;
    }
}

}  // namespace

extern "C" int vr_select_threshold(const uint64_t* d_hist, const uint64_t* d_hist_top, int rule,
                                   int param, uint32_t* d_result, uint32_t* d_keep_bits,
                                   void* stream)
{
    vr::clear_error();
    VR_REQUIRE(d_hist && d_result && d_keep_bits, VR_ERR_NULL, "vr_select_threshold: NULL pointer");
    VR_REQUIRE(rule >= VR_RULE_VALLEY && rule <= VR_RULE_NONE, VR_ERR_RANGE,
               "vr_select_threshold: unknown rule %d", rule);
    if (rule == VR_RULE_VALLEY)
        VR_REQUIRE(param >= 1 && param <= 4096, VR_ERR_RANGE,
                   "vr_select_threshold: smoothing radius %d outside [1, 4096]", param);
    if (rule == VR_RULE_OTSU || rule == VR_RULE_ITS)
        VR_REQUIRE(param >= 0 && param <= 12, VR_ERR_RANGE,
                   "vr_select_threshold: bin width shift %d outside [0, 12]", param);
    select_kernel<<<1, kT, 0, vr::as_stream(stream)>>>(d_hist, d_hist_top, rule, param, d_result,
                                                       d_keep_bits);
    return vr::check_launch("vr_select_threshold");
}

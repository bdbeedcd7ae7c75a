// Threshold selection and keep mask on the device (Sections III-A and III-D).
//
// Four launches on the caller's stream.  The histogram is cut into chunks of
// 1024 bins; a chunk workgroup (one bin per thread) loads its bins plus a halo
// with coalesced reads and works from a block scan in LDS.
//   1. per chunk: the chunk's maximum of the smoothed histogram (valley), or
//      its count and grey-value sum (Otsu, ITS);
//   2. per chunk: valley candidates against the global peak, or the chunk's
//      best Otsu threshold;
//   3. one workgroup: combines the chunks (runs the ITS iteration) and writes
//      the result;
//   4. one workgroup per 1024 bins: the keep mask from the threshold.
// The caller's keep-mask buffer (8 KiB) carries the per-chunk records between
// the launches and is overwritten with the mask at the end, so nothing is
// allocated.  Floating point that decides a threshold uses IEEE FP64
// operations written out one by one, in the order stated for each rule.
#include "select_dev.h"

namespace {

using namespace vr::sel;

__global__ void __launch_bounds__(kT)
chunk_pass_kernel(const uint64_t* __restrict__ H, int rule, int param, uint32_t* __restrict__ scratch)
{
    __shared__ SelLds Ls;
    chunk_pass(Ls, (int)blockIdx.x, H, rule, param, scratch);
}

__global__ void __launch_bounds__(kT)
chunk_search_kernel(const uint64_t* __restrict__ H, int rule, int param, int n_chunks,
                    uint32_t* __restrict__ scratch)
{
    __shared__ SelLds Ls;
    chunk_search(Ls, (int)blockIdx.x, H, rule, param, n_chunks, scratch);
}

__global__ void __launch_bounds__(kT)
finish_kernel(const uint64_t* __restrict__ H, const uint64_t* __restrict__ Htop, int rule, int param,
              int n_chunks, uint32_t* __restrict__ result, uint32_t* __restrict__ bits)
{
    __shared__ SelLds Ls;
    finish(Ls, H, Htop, rule, param, n_chunks, result, bits, false);
}

// row blockIdx.x of the keep mask, from the threshold the finish launch wrote
__global__ void __launch_bounds__(kT)
mask_kernel(const uint64_t* __restrict__ Htop, const uint32_t* __restrict__ result, uint32_t* __restrict__ bits)
{
    mask_row(Htop, result[0], (int)blockIdx.x, bits);
}

}  // namespace

extern "C" int vr_select_threshold(const uint64_t* d_hist, const uint64_t* d_hist_top, int rule,
                                   int param, uint32_t* d_result, uint32_t* d_keep_bits,
                                   void* stream)
{
    vr::clear_error();
    VR_REQUIRE(d_hist && d_result && d_keep_bits, VR_ERR_NULL, "vr_select_threshold: NULL pointer");
    VR_REQUIRE((reinterpret_cast<uintptr_t>(d_hist) & 15u) == 0, VR_ERR_RANGE,
               "vr_select_threshold: d_hist must be 16-byte aligned");
    VR_REQUIRE(rule >= VR_RULE_VALLEY && rule <= VR_RULE_NONE, VR_ERR_RANGE,
               "vr_select_threshold: unknown rule %d", rule);
    if (rule == VR_RULE_VALLEY)
        VR_REQUIRE(param >= 1 && param <= kMaxRadius, VR_ERR_RANGE,
                   "vr_select_threshold: smoothing radius %d outside [1, %d]", param, kMaxRadius);
    if (rule == VR_RULE_OTSU || rule == VR_RULE_ITS)
        VR_REQUIRE(param >= 0 && param <= 12, VR_ERR_RANGE,
                   "vr_select_threshold: bin width shift %d outside [0, 12]", param);
    hipStream_t s = vr::as_stream(stream);
    const int bins = rule == VR_RULE_VALLEY ? kB : (kB >> param);
    const int n_chunks = (bins + kT - 1) / kT;
    if (rule != VR_RULE_NONE) {
        chunk_pass_kernel<<<n_chunks, kT, 0, s>>>(d_hist, rule, param, d_keep_bits);
        int rc = vr::check_launch("vr_select_threshold: chunk pass");
        if (rc) return rc;
        if (rule != VR_RULE_ITS) {
            chunk_search_kernel<<<n_chunks, kT, 0, s>>>(d_hist, rule, param, n_chunks, d_keep_bits);
            rc = vr::check_launch("vr_select_threshold: chunk search");
            if (rc) return rc;
        }
    }
    finish_kernel<<<1, kT, 0, s>>>(d_hist, d_hist_top, rule, param, n_chunks, d_result, d_keep_bits);
    int rc = vr::check_launch("vr_select_threshold: finish");
    if (rc) return rc;
    mask_kernel<<<kB / kT, kT, 0, s>>>(d_hist_top, d_result, d_keep_bits);
    return vr::check_launch("vr_select_threshold");
}

// Instantiation of the 16-bit MFMA Strassen kernels: fp32 operands in the compensated bf16x3 mode, A and B as stored.
#include "gemm_mfma16.hpp"

namespace strassen {

hipError_t launch_m16_bf16x3_nn(bool large, int wa, int wb, int wc, const LaunchArgs &a, int batch, bool vec,
                                hipStream_t s) {
    return large ? m16k::dispatch<m16k::LargeX3, m16k::X3Ops, true, false>(wa, wb, wc, a, batch, vec, s)
                 : m16k::dispatch<m16k::Small, m16k::X3Ops, true, false>(wa, wb, wc, a, batch, vec, s);
}

hipError_t launch_m16_bf16x3_chained(const LaunchArgs &a, int nchains, bool vec, hipStream_t s) {
    return m16k::launch_chained<m16k::TileFor<m16k::LargeX3, m16k::X3Ops, 1, 1, true, false>, m16k::X3Ops>(a, nchains, vec, s);
}

}  // namespace strassen

// Instantiation of the 16-bit MFMA Strassen kernels: bf16 operands.
#include "gemm_mfma16.hpp"

namespace strassen {

hipError_t launch_m16_bf16(bool large, int wa, int wb, int wc, const LaunchArgs &a, int batch, bool vec,
                           hipStream_t s) {
    return large ? m16k::dispatch<m16k::Large, m16k::Bf16Ops, true, false>(wa, wb, wc, a, batch, vec, s)
                 : m16k::dispatch<m16k::Small, m16k::Bf16Ops, true, false>(wa, wb, wc, a, batch, vec, s);
}

hipError_t launch_m16_bf16_chained(const LaunchArgs &a, int nchains, bool vec, hipStream_t s) {
    return m16k::launch_chained<m16k::TileFor<m16k::Large, m16k::Bf16Ops, 1, 1>, m16k::Bf16Ops>(a, nchains, vec, s);
}

}  // namespace strassen

// Instantiation of the 16-bit MFMA Strassen kernels for fp32 operands in the compensated bf16x3 mode.
#include "gemm_mfma16.hpp"

namespace strassen {

hipError_t launch_m16_bf16x3(int wa, int wb, int wc, const LaunchArgs &a, int batch, bool vec,
                        hipStream_t s) {
    return dispatch<X3Ops>(wa, wb, wc, a, batch, vec, s);
}

}  // namespace strassen

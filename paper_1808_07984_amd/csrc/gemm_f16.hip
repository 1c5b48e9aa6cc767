// Instantiation of the 16-bit MFMA Strassen kernels for fp16 operands.
#include "gemm_mfma16.hpp"

namespace strassen {

hipError_t launch_m16_f16(int wa, int wb, int wc, const LaunchArgs &a, int batch, bool vec,
                        hipStream_t s) {
    return dispatch<F16Ops>(wa, wb, wc, a, batch, vec, s);
}

}  // namespace strassen

// Instantiation of the 16-bit MFMA Strassen kernels for bf16 operands (and the 16-bit path dispatcher).
#include "gemm_mfma16.hpp"

namespace strassen {

hipError_t launch_m16_bf16(int wa, int wb, int wc, const LaunchArgs &a, int batch, bool vec,
                        hipStream_t s) {
    return dispatch<Bf16Ops>(wa, wb, wc, a, batch, vec, s);
}

KernelShape m16_tile_shape(bool x3) {
    // 16-byte loads cover 8 elements of a 16-bit type, 4 fp32 (x3 loads two).
    return KernelShape{M16Tile::MT, M16Tile::NT, M16Tile::KT, x3 ? 4 : 8};
}

hipError_t launch_m16(Operand16 op, int wa, int wb, int wc, const LaunchArgs &a, int batch,
                      bool vec, hipStream_t s) {
    switch (op) {
        case Operand16::kBf16: return launch_m16_bf16(wa, wb, wc, a, batch, vec, s);
        case Operand16::kF16: return launch_m16_f16(wa, wb, wc, a, batch, vec, s);
        case Operand16::kBf16x3: return launch_m16_bf16x3(wa, wb, wc, a, batch, vec, s);
    }
    return hipErrorInvalidValue;
}

const char *m16_kernel_name(Operand16 op) {
    switch (op) {
        case Operand16::kBf16: return "strassen_m16_kernel<bf16>";
        case Operand16::kF16: return "strassen_m16_kernel<f16>";
        case Operand16::kBf16x3: return "strassen_m16_kernel<bf16x3>";
    }
    return "strassen_m16_kernel";
}

}  // namespace strassen

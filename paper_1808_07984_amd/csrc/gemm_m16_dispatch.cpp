// Host-side selection among the 16-bit MFMA kernel instantiations.
#include "launch.hpp"

namespace strassen {

KernelShape m16_tile_shape(bool x3, bool large, int wa, int wb, bool untransposed) {
    // 16-byte loads cover 8 elements of a 16-bit type or 4 fp32.  k-tile of
    // the large tiles by operand terms: 16-bit 64 up to four in all, 32
    // above and for (1,2,2); compensated 32 for the untransposed
    // single-term product, 16 otherwise.
    if (large) {
        const int terms = wa + wb;
        const int kt = x3 ? (terms == 2 && untransposed ? 32 : 16)
                          : (terms <= 4 && !(wa == 1 && wb == 2) ? 64 : 32);
        return KernelShape{256, 256, kt, x3 ? 4 : 8};
    }
    return KernelShape{128, 128, 32, x3 ? 4 : 8};
}

hipError_t launch_m16(Operand16 op, bool trans_a, bool trans_b, bool large, int wa, int wb, int wc,
                      const LaunchArgs &a, int batch, bool vec, hipStream_t s) {
    switch (op) {
        case Operand16::kBf16:
            if (trans_a || trans_b) return hipErrorInvalidValue;
            return launch_m16_bf16(large, wa, wb, wc, a, batch, vec, s);
        case Operand16::kF16:
            if (trans_a || trans_b) return hipErrorInvalidValue;
            return launch_m16_f16(large, wa, wb, wc, a, batch, vec, s);
        case Operand16::kBf16x3:
            if (!trans_a && !trans_b) return launch_m16_bf16x3_nn(large, wa, wb, wc, a, batch, vec, s);
            if (!trans_a && trans_b) return launch_m16_bf16x3_nt(large, wa, wb, wc, a, batch, vec, s);
            if (trans_a && !trans_b) return launch_m16_bf16x3_tn(large, wa, wb, wc, a, batch, vec, s);
            return launch_m16_bf16x3_tt(large, wa, wb, wc, a, batch, vec, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_m16_chained(Operand16 op, const LaunchArgs &a, int nchains, bool vec, hipStream_t s) {
    switch (op) {
        case Operand16::kBf16: return launch_m16_bf16_chained(a, nchains, vec, s);
        case Operand16::kF16: return launch_m16_f16_chained(a, nchains, vec, s);
        case Operand16::kBf16x3: return launch_m16_bf16x3_chained(a, nchains, vec, s);
    }
    return hipErrorInvalidValue;
}

const char *m16_kernel_name(Operand16 op, bool large) {
    switch (op) {
        case Operand16::kBf16: return large ? "strassen_m16_kernel<bf16,256x256>" : "strassen_m16_kernel<bf16,128x128>";
        case Operand16::kF16: return large ? "strassen_m16_kernel<f16,256x256>" : "strassen_m16_kernel<f16,128x128>";
        case Operand16::kBf16x3: return large ? "strassen_m16_kernel<bf16x3,256x256>" : "strassen_m16_kernel<bf16x3,128x128>";
    }
    return "strassen_m16_kernel";
}

const char *m16_x3pre_kernel_name(bool pre_b, bool large) {
    if (pre_b) return large ? "strassen_m16_kernel<bf16x3p,256x256>" : "strassen_m16_kernel<bf16x3p,128x128>";
    return large ? "strassen_m16_kernel<bf16x3pa,256x256>" : "strassen_m16_kernel<bf16x3pa,128x128>";
}

}  // namespace strassen

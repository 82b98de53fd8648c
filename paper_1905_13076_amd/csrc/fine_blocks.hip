// Register-row fine kernels with 256- and 512-thread workgroups: the autotuner's other
// candidates next to the 1024-thread forms of fine.hip (same device code, fine_chain.hpp).
// A smaller workgroup takes more rows per thread (R = 1, 2, 4, 8) and synchronises fewer
// waves per PCG reduction; whether that pays depends on the mesh and is measured.
#include "fine_chain.hpp"

namespace ppc {

namespace {

template <typename S, int R, int B>
void launch_one(const FineArgs& a, int N, size_t lds, hipStream_t s) {
    static bool attr_set = false;
    if (!attr_set) {
        PPC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fine_sweep<S, R, B, 0>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget));
        attr_set = true;
    }
    hipLaunchKernelGGL((k_fine_sweep<S, R, B, 0>), dim3(N), dim3(B), lds, s, a);
}

template <typename S, int R, int B>
void launch_batch_one(const FineArgs* args, const int2* work, int nblocks, size_t lds, hipStream_t s) {
    static bool attr_set = false;
    if (!attr_set) {
        PPC_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fine_sweep_batch<S, R, B, 0>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBudget));
        attr_set = true;
    }
    hipLaunchKernelGGL((k_fine_sweep_batch<S, R, B, 0>), dim3(nblocks), dim3(B), lds, s, args, work);
}

template <typename S, int B>
void rows_typed(const FineArgs& a, int N, const FineShape& sh, hipStream_t s) {
    switch (sh.R) {
        case 1: launch_one<S, 1, B>(a, N, sh.lds, s); break;
        case 2: launch_one<S, 2, B>(a, N, sh.lds, s); break;
        case 4: launch_one<S, 4, B>(a, N, sh.lds, s); break;
        case 8: launch_one<S, 8, B>(a, N, sh.lds, s); break;
        default: fail(PPC_ERR_ARG, "no register-row kernel with R = " + std::to_string(sh.R));
    }
}

template <typename S, int B>
void rows_batch_typed(const FineArgs* args, const int2* work, int nblocks, const FineShape& sh, hipStream_t s) {
    switch (sh.R) {
        case 1: launch_batch_one<S, 1, B>(args, work, nblocks, sh.lds, s); break;
        case 2: launch_batch_one<S, 2, B>(args, work, nblocks, sh.lds, s); break;
        case 4: launch_batch_one<S, 4, B>(args, work, nblocks, sh.lds, s); break;
        case 8: launch_batch_one<S, 8, B>(args, work, nblocks, sh.lds, s); break;
        default: fail(PPC_ERR_ARG, "no register-row kernel with R = " + std::to_string(sh.R));
    }
}

}  // namespace

void launch_fine_rows_small(const FineArgs& a, int N, const FineShape& sh, bool fp64, hipStream_t s) {
    if (sh.block == 512) {
        if (fp64) rows_typed<double, 512>(a, N, sh, s);
        else rows_typed<float, 512>(a, N, sh, s);
    } else if (sh.block == 256) {
        if (fp64) rows_typed<double, 256>(a, N, sh, s);
        else rows_typed<float, 256>(a, N, sh, s);
    } else {
        fail(PPC_ERR_ARG, "no register-row kernel with " + std::to_string(sh.block) + " threads");
    }
}

void launch_fine_batch_rows_small(const FineArgs* args, const int2* work, int nblocks, const FineShape& sh,
                                  bool fp64, hipStream_t s) {
    if (sh.block == 512) {
        if (fp64) rows_batch_typed<double, 512>(args, work, nblocks, sh, s);
        else rows_batch_typed<float, 512>(args, work, nblocks, sh, s);
    } else if (sh.block == 256) {
        if (fp64) rows_batch_typed<double, 256>(args, work, nblocks, sh, s);
        else rows_batch_typed<float, 256>(args, work, nblocks, sh, s);
    } else {
        fail(PPC_ERR_ARG, "no register-row kernel with " + std::to_string(sh.block) + " threads");
    }
}

}  // namespace ppc

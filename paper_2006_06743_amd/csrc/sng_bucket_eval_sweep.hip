// Partner-block evaluate kernels for the sweep (level codes and histograms).
#include "sng_bucket_eval.hpp"

namespace sng {

hipError_t launch_bucket_eval_sweep(const Inst &I, const SweepArgs &S, const BucketGeom &B,
                                    const PassAShape &sh, hipStream_t st)
{
    if (B.lds) {
        const size_t lds = ((size_t)1 << B.bshift) * (size_t)I.d * sizeof(float);
        const bool buf = use_buffer(I), lr = lane_rows_fit(I);
        return dispatch_small_d(I.d, [&]<int D>() -> hipError_t {
#define SNG_LDS_LAUNCH(BUF, LR)                                                              \
    hipLaunchKernelGGL((k_bkt_eval_lds_sweep<D, BUF, LR>), dim3(compute_units()),           \
                       dim3(kLdsThreads), lds, st, I, B, S)
            if (buf && lr) SNG_LDS_LAUNCH(true, true);
            else if (buf) SNG_LDS_LAUNCH(true, false);
            else if (lr) SNG_LDS_LAUNCH(false, true);
            else SNG_LDS_LAUNCH(false, false);
#undef SNG_LDS_LAUNCH
            return hipGetLastError();
        });
    }
    const bool vec_ok = ((uintptr_t)I.X % 16 == 0) && (I.ld % 4 == 0);
    return dispatch(I.d, vec_ok, sh, [&]<class Row, int OB>(uint32_t) -> hipError_t {
        if constexpr (Row::kPrefetch) {
            if (use_buffer(I))
                hipLaunchKernelGGL((k_bkt_eval_sweep<Row, OB, true>), dim3(eval_blocks(B)),
                                   dim3(256), 0, st, I, B, S);
            else
                hipLaunchKernelGGL((k_bkt_eval_sweep<Row, OB, false>), dim3(eval_blocks(B)),
                                   dim3(256), 0, st, I, B, S);
            return hipGetLastError();
        } else {
            return hipErrorInvalidValue;
        }
    });
}

}  // namespace sng

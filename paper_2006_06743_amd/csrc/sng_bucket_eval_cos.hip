// Partner-block evaluate kernels for the cosine query.
#include "sng_bucket_eval.hpp"

namespace sng {

template hipError_t launch_bucket_eval<kSimCos>(const Inst &, const BucketGeom &, const PassAShape &,
                                           hipStream_t);

}  // namespace sng

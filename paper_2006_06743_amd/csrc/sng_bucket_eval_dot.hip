// Partner-block evaluate kernels for the dot-product query.
#include "sng_bucket_eval.hpp"

namespace sng {

template hipError_t launch_bucket_eval<kSimDot>(const Inst &, const BucketGeom &, const PassAShape &,
                                           hipStream_t);

}  // namespace sng

// Partner-block evaluate kernels for the distance query (the plain pass).
#include "sng_bucket_eval.hpp"

namespace sng {

template hipError_t launch_bucket_eval<kSimNone>(const Inst &, const BucketGeom &, const PassAShape &,
                                           hipStream_t);

}  // namespace sng

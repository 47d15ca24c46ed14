// Step kernels with exactly one tile per block, instantiated for FP64 storage
// (a translation unit of their own, so that both sets compile in parallel).
#include "lbm_lattice_impl.h"

namespace lbm {

bool launch_lattice_fp64_one(const Geom& G, int mode, int variant, const void* src, void* dst, BoxDev* boxes,
                          const int* toff, const int* tlist, const void* rec, double* out0, double* out1,
                          const unsigned long long* tin, unsigned long long* tout, hipStream_t s, hipEvent_t ev0,
                          hipEvent_t ev1)
{
    return launch_lattice_s<ST_FP64, true>(G, mode, variant, src, dst, boxes, toff, tlist, rec, out0, out1, tin, tout, s,
                                         ev0, ev1);
}

}  // namespace lbm

// Lattice kernels instantiated for FP64 population storage.
#include "lbm_lattice_impl.h"

namespace lbm {

// step kernels with one tile per block (lbm_lattice_fp64_one.hip)
bool launch_lattice_fp64_one(const Geom& G, int mode, int variant, const void* src, void* dst, BoxDev* boxes,
                          const int* toff, const int* tlist, const void* rec, double* out0, double* out1,
                          const unsigned long long* tin, unsigned long long* tout, hipStream_t s, hipEvent_t ev0,
                          hipEvent_t ev1);

bool launch_lattice_fp64(const Geom& G, int mode, int variant, const void* src, void* dst, BoxDev* boxes, const int* toff,
                          const int* tlist, const void* rec, double* out0, double* out1, const unsigned long long* tin,
                          unsigned long long* tout, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    if (mode == M_STEP && (variant & 128) && G.tpb == 1)
        return launch_lattice_fp64_one(G, mode, variant, src, dst, boxes, toff, tlist, rec, out0, out1, tin, tout, s, ev0,
                                      ev1);
    return launch_lattice_s<ST_FP64, false>(G, mode, variant, src, dst, boxes, toff, tlist, rec, out0, out1, tin, tout, s,
                                          ev0, ev1);
}

}  // namespace lbm

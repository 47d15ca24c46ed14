// Lattice entry points: storage dispatch of the step / moment / diagnostic
// kernels (instantiated in lbm_lattice_<storage>.hip from lbm_lattice_impl.h),
// the equilibrium initialisation and the tile shapes they support.
#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

bool launch_lattice_fp64(const Geom& G, int mode, int variant, const void* src, void* dst, BoxDev* boxes, const int* toff,
                          const int* tlist, const void* rec, double* out0, double* out1, const unsigned long long* tin,
                          unsigned long long* tout, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
bool launch_lattice_fp32(const Geom& G, int mode, int variant, const void* src, void* dst, BoxDev* boxes, const int* toff,
                          const int* tlist, const void* rec, double* out0, double* out1, const unsigned long long* tin,
                          unsigned long long* tout, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
bool launch_lattice_fp16(const Geom& G, int mode, int variant, const void* src, void* dst, BoxDev* boxes, const int* toff,
                          const int* tlist, const void* rec, double* out0, double* out1, const unsigned long long* tin,
                          unsigned long long* tout, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
bool launch_lattice_mom32(const Geom& G, int mode, int variant, const void* src, void* dst, BoxDev* boxes, const int* toff,
                          const int* tlist, const void* rec, double* out0, double* out1, const unsigned long long* tin,
                          unsigned long long* tout, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);

// Equilibrium of Eq. eqf at (rho, u) written so that the next pull sees it at
// every node: the copy held at node y for population i is the equilibrium of
// node y + c_i.
template <int ST>
__global__ __launch_bounds__(BLOCK) void k_equilibrium(const Geom G, typename StoreT<ST>::S* __restrict__ dst,
                                                       const BoxDev* __restrict__ boxes,
                                                       const double* __restrict__ rho, const double* __restrict__ u)
{
    using S = typename StoreT<ST>::S;
    const long long gid = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (gid >= G.N * G.nboxes) return;
    const int box = int(gid / G.N);
    const long long n = gid % G.N;
    const int x = int(n % G.nx), y = int((n / G.nx) % G.ny), z = int(n / ((long long)G.nx * G.ny));
    const long long row = n / G.nx;
    const double s = ST == ST_FP16 ? ldexp(1.0, boxes[box].e_data) : 1.0;
    S* db = dst + (long long)box * G.sbox;
    if constexpr (ST == ST_MOM32) {
        // the equilibrium of this node taken as its post-collision state
        const double r = rho[(long long)box * G.N + n];
        const double v[3] = {u[((long long)box * 3 + 0) * G.N + n], u[((long long)box * 3 + 1) * G.N + n],
                             u[((long long)box * 3 + 2) * G.N + n]};
        const double uu = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        const double piece[MP_N] = {(r - G.rho0) - 1.5 * r * uu, 3 * r * v[0], 3 * r * v[1], 3 * r * v[2],
                                    4.5 * r * v[0] * v[0], 4.5 * r * v[1] * v[1], 4.5 * r * v[2] * v[2],
                                    9 * r * v[0] * v[1], 9 * r * v[0] * v[2], 9 * r * v[1] * v[2]};
        for (int k = 0; k < MP_N; ++k) db[pop_index(G.rb, G.kp, k, row, x)] = S(piece[k]);
        return;
    }
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        int xs = x + cvel(i, 0), ys = y + cvel(i, 1), zs = z + cvel(i, 2);
        xs = xs < 0 ? xs + G.nx : (xs >= G.nx ? xs - G.nx : xs);
        ys = ys < 0 ? ys + G.ny : (ys >= G.ny ? ys - G.ny : ys);
        zs = zs < 0 ? zs + G.nz : (zs >= G.nz ? zs - G.nz : zs);
        const long long m = ((long long)zs * G.ny + ys) * G.nx + xs;
        const double r = rho[(long long)box * G.N + m];
        const double vx = u[((long long)box * 3 + 0) * G.N + m];
        const double vy = u[((long long)box * 3 + 1) * G.N + m];
        const double vz = u[((long long)box * 3 + 2) * G.N + m];
        const double cu = cvel(i, 0) * vx + cvel(i, 1) * vy + cvel(i, 2) * vz;
        const double uu = vx * vx + vy * vy + vz * vz;
        const double bracket = (r - G.rho0) + 3.0 * r * cu + 4.5 * r * (cu * cu - uu / 3.0);
        db[pop_index(G.rb, G.kp, i, row, x)] = ST == ST_FP16 ? S(bracket * s) : S(wgt(i) * bracket);
    }
}

bool tile_supported(int tx, int ty, int tz)
{
    const int ok[][3] = {{64, 2, 2}, {64, 4, 1}, {64, 1, 4}, {32, 4, 2}, {32, 2, 4},
                         {16, 4, 4}, {128, 2, 1}, {128, 1, 2}, {256, 1, 1}};
    for (auto& o : ok)
        if (o[0] == tx && o[1] == ty && o[2] == tz) return true;
    return false;
}

bool launch_lattice(int storage, const Geom& G, int mode, int variant, const void* src, void* dst, BoxDev* boxes,
                    const int* toff, const int* tlist, const void* rec, double* out0, double* out1,
                    const unsigned long long* tin, unsigned long long* tout, hipStream_t s, hipEvent_t ev0,
                    hipEvent_t ev1)
{
    switch (storage) {
    case ST_FP64:
        return launch_lattice_fp64(G, mode, variant, src, dst, boxes, toff, tlist, rec, out0, out1, tin, tout, s, ev0,
                                   ev1);
    case ST_FP32:
        return launch_lattice_fp32(G, mode, variant, src, dst, boxes, toff, tlist, rec, out0, out1, tin, tout, s, ev0,
                                   ev1);
    case ST_FP16:
        return launch_lattice_fp16(G, mode, variant, src, dst, boxes, toff, tlist, rec, out0, out1, tin, tout, s, ev0,
                                   ev1);
    case ST_MOM32:
        return launch_lattice_mom32(G, mode, variant, src, dst, boxes, toff, tlist, rec, out0, out1, tin, tout, s, ev0,
                                    ev1);
    }
    return false;
}

void launch_equilibrium(int storage, const Geom& G, void* dst, const BoxDev* boxes, const double* rho,
                        const double* u, hipStream_t s)
{
    const long long total = G.N * G.nboxes;
    const unsigned nb = (unsigned)((total + BLOCK - 1) / BLOCK);
    switch (storage) {
    case ST_FP64:
        hipLaunchKernelGGL(k_equilibrium<ST_FP64>, dim3(nb), dim3(BLOCK), 0, s, G, (double*)dst, boxes, rho, u);
        break;
    case ST_FP32:
        hipLaunchKernelGGL(k_equilibrium<ST_FP32>, dim3(nb), dim3(BLOCK), 0, s, G, (float*)dst, boxes, rho, u);
        break;
    case ST_FP16:
        hipLaunchKernelGGL(k_equilibrium<ST_FP16>, dim3(nb), dim3(BLOCK), 0, s, G, (_Float16*)dst, boxes, rho, u);
        break;
    case ST_MOM32:
        hipLaunchKernelGGL(k_equilibrium<ST_MOM32>, dim3(nb), dim3(BLOCK), 0, s, G, (float*)dst, boxes, rho, u);
        break;
    }
}

}  // namespace lbm

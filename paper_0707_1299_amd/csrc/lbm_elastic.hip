// Marker forces of singular curves and surfaces (Sec. I; Eq. singularF with a
// line or area measure): Hookean bead-spring chains and closed triangulated
// interfaces with tension.  One thread per marker; each marker gathers its
// own contributions (springs to its chain neighbours, or the area gradients
// of its incident triangles in incidence order), so the sums are
// deterministic.  Distances are taken as the nearest periodic image.
#include <math.h>

#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

namespace {

__device__ __forceinline__ double min_image(double d, double L) { return d - L * rint(d / L); }

__device__ __forceinline__ void load3(const double* p, long long i, double (&v)[3])
{
    v[0] = p[3 * i];
    v[1] = p[3 * i + 1];
    v[2] = p[3 * i + 2];
}

__device__ __forceinline__ void cross(const double (&a)[3], const double (&b)[3], double (&c)[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

__global__ __launch_bounds__(256) void k_chain_forces(const Geom G, long long n, int m, double k, double l0,
                                                      const double* __restrict__ pos, const double* __restrict__ ext,
                                                      double* __restrict__ frc)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double L[3] = {double(G.nx), double(G.ny), double(G.nz)};
    double r[3], F[3] = {0.0, 0.0, 0.0};
    load3(pos, i, r);
    if (ext) load3(ext, i, F);
    // spring to the next marker of the chain, then the one from the previous marker
    for (int side = 0; side < 2; ++side) {
        const bool has = side == 0 ? (i + 1) % m != 0 : i % m != 0;
        if (!has) continue;
        const long long j = side == 0 ? i + 1 : i - 1;
        double q[3], d[3];
        load3(pos, j, q);
        for (int a = 0; a < 3; ++a) d[a] = min_image(side == 0 ? q[a] - r[a] : r[a] - q[a], L[a]);
        const double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double s = k * (len - l0) / len;
        for (int a = 0; a < 3; ++a) F[a] += side == 0 ? s * d[a] : -(s * d[a]);
    }
    for (int a = 0; a < 3; ++a) frc[3 * i + a] = F[a];
}

__global__ __launch_bounds__(256) void k_surface_forces(const Geom G, long long n, double gamma,
                                                        const double* __restrict__ pos, const double* __restrict__ ext,
                                                        const int* __restrict__ tri, const int* __restrict__ vt_off,
                                                        const int* __restrict__ vt_idx, double* __restrict__ frc)
{
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const double L[3] = {double(G.nx), double(G.ny), double(G.nz)};
    double F[3] = {0.0, 0.0, 0.0};
    if (ext) load3(ext, v, F);
    for (int e = vt_off[v]; e < vt_off[v + 1]; ++e) {
        const int t = vt_idx[e];
        const int ia = tri[3 * t], ib = tri[3 * t + 1], ic = tri[3 * t + 2];
        double pa[3], pb[3], pc[3];
        load3(pos, ia, pa);
        load3(pos, ib, pb);
        load3(pos, ic, pc);
        double ab[3], ac[3];
        for (int a = 0; a < 3; ++a) {
            pb[a] = pa[a] + min_image(pb[a] - pa[a], L[a]);
            pc[a] = pa[a] + min_image(pc[a] - pa[a], L[a]);
            ab[a] = pb[a] - pa[a];
            ac[a] = pc[a] - pa[a];
        }
        double nrm[3];
        cross(ab, ac, nrm);
        const double il = 1.0 / sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
        for (int a = 0; a < 3; ++a) nrm[a] *= il;
        // dA/dv = n x (opposite edge, in the triangle's orientation) / 2
        double edge[3];
        for (int a = 0; a < 3; ++a)
            edge[a] = v == ia ? pc[a] - pb[a] : (v == ib ? pa[a] - pc[a] : pb[a] - pa[a]);
        double g[3];
        cross(nrm, edge, g);
        for (int a = 0; a < 3; ++a) F[a] -= gamma * (0.5 * g[a]);
    }
    for (int a = 0; a < 3; ++a) frc[3 * v + a] = F[a];
}

unsigned nblk(long long n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

void launch_elastic_forces(const Geom& G, const ElasticLaunch& e, hipStream_t s)
{
    if (e.n <= 0) return;
    if (e.kind == 0)
        hipLaunchKernelGGL(k_chain_forces, dim3(nblk(e.n, 256)), dim3(256), 0, s, G, e.n, e.chain_len, e.k_spring,
                           e.l0, e.pos, e.ext, e.frc);
    else
        hipLaunchKernelGGL(k_surface_forces, dim3(nblk(e.n, 256)), dim3(256), 0, s, G, e.n, e.tension, e.pos, e.ext,
                           e.tri, e.vt_off, e.vt_idx, e.frc);
}

}  // namespace lbm

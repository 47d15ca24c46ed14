// Host-side declarations shared by the liblbm translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_device.h"

namespace lbm {

constexpr int LBD_N = 13;               // diagnostics per box
constexpr int LBML_NPARAM_DEV = 4545;   // MLP parameters

struct AdvectLaunch {
    long long n, off;
    const double* frc;
    double* pos;
    double* vel_out;
    double* vel_sum;
    const int* boxid;
    double inv_a, inv_aL;
    const uint16_t* mlp;
    float in_shift[4], in_scale[4], out_scale;
    int advect;
    const unsigned long long* tin;   // thermal runs: step counter of this step (else NULL)
};

// marker forces of a chain (kind 0) or surface (kind 1) set
struct ElasticLaunch {
    int kind;
    int chain_len;
    long long n;
    const double* pos;
    const double* ext;
    double* frc;
    double k_spring, l0, tension;
    const int* tri;
    const int* vt_off;
    const int* vt_idx;
};

bool tile_supported(int tx, int ty, int tz);
void launch_elastic_forces(const Geom& G, const ElasticLaunch& e, hipStream_t s);
bool launch_lattice(int storage, const Geom& G, int mode, int variant, const void* src, void* dst, BoxDev* boxes,
                    const int* toff, const int* tlist, const void* rec, double* out0, double* out1,
                    const unsigned long long* tin, unsigned long long* tout, hipStream_t s, hipEvent_t ev0 = nullptr,
                    hipEvent_t ev1 = nullptr);
void launch_equilibrium(int storage, const Geom& G, void* dst, const BoxDev* boxes, const double* rho,
                        const double* u, hipStream_t s);

void launch_fill_u32(void* p, long long n, uint32_t v, hipStream_t s);
long long prep_blocks(long long n);
void launch_prep(int storage, const Geom& G, long long n, long long off, const double* pos, const double* frc,
                 const int* boxid, void* rec, int* err, double* psum, hipStream_t s);
long long scan_blocks(long long ntiles);
void launch_bins(int storage, const Geom& G, long long npts, const void* rec, int* count, int* bsum, int* toff,
                 int* cursor, int* tlist, int* tlist_tmp, int* err, hipStream_t s);
void launch_box_update(int storage, const Geom& G, const void* rec, const int* toff, const int* tlist,
                       const double* psum, long long npsum, const float* tmax, double* part, float* pmax,
                       unsigned* ticket, BoxDev* boxes, int zero_net, int fp16_exp, hipStream_t s);
void launch_advect(int storage, const Geom& G, const AdvectLaunch& a, const BoxDev* boxes, void* partial,
                   hipStream_t s);
void launch_interp_points(int storage, const Geom& G, long long n, const double* pos, const int* boxid, double* out,
                          const void* src, const BoxDev* boxes, const int* toff, const int* tlist, const void* rec,
                          hipStream_t s);
void launch_diag_reduce(const Geom& G, const double* part, double* out, hipStream_t s);

}  // namespace lbm

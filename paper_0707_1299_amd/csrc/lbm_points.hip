// Point-force kernels: per-point stencil records, deterministic binning of
// points to the lattice tiles of a window around their stencils (rebuilt only
// when a stencil leaves its window), per-box force sums and
// FP16 exponents, the colloid update, interpolation at arbitrary points and
// the reduction of the diagnostics.
//
// Spreading and interpolation use Peskin's 4-point kernel (Eq. deltadef,
// Sec. III) over the 4x4x4 nodes floor(R)-1 .. floor(R)+2 of each point.
// The colloid update is dR/dt = v(R) + F/(6 pi eta) (1/a - 1/a_L) (Sec. IV),
// integrated with one explicit Euler step per lattice step.
#include <math.h>

#include <algorithm>

#include "lbm_device.h"
#include "lbm_internal.h"
#include "lbm_noise.h"

namespace lbm {

// Binning window: a point is binned to the tiles met by WIN = 5 consecutive nodes
// per axis, starting at its window base.  The 4-node Peskin stencil of the point
// (base floor(R) - 1) lies in the window while base - window base is 0 or 1
// (periodic), so the tile lists stay valid as the point moves, until a stencil
// leaves its window ("skin crossing"); only then are the lists rebuilt.  The
// window base is chosen when binning so that the point can move at least half a
// node either way first: one node below the stencil base when the point sits in
// the lower half of its cell, at the stencil base otherwise.
constexpr int WIN = 5;

// Distinct tiles met by the WIN consecutive nodes base .. base+WIN-1 (periodic) of
// one axis, in order of first appearance.
__device__ __forceinline__ int axis_tiles(int base, int n, int lt, int (&out)[WIN])
{
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < WIN; ++k) {
        int node = base + k;
        if (node >= n) node -= n;
        const int t = node >> lt;
        bool dup = false;
        for (int j = 0; j < cnt; ++j) dup |= (out[j] == t);
        if (!dup) out[cnt++] = t;
    }
    return cnt;
}

// number of distinct tiles met by the window (as axis_tiles, without the list: every index
// is known at compile time, so nothing goes to scratch memory)
__device__ __forceinline__ int axis_count(int base, int n, int lt)
{
    int t[WIN];
#pragma unroll
    for (int k = 0; k < WIN; ++k) {
        int node = base + k;
        if (node >= n) node -= n;
        t[k] = node >> lt;
    }
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < WIN; ++k) {
        bool dup = false;
#pragma unroll
        for (int j = 0; j < k; ++j) dup |= (t[j] == t[k]);
        cnt += dup ? 0 : 1;
    }
    return cnt;
}

struct TileSet {
    int tx[WIN], ty[WIN], tz[WIN];
    int cx, cy, cz;
};

// tiles of the window with bases (wx, wy, wz)
__device__ __forceinline__ void window_tiles(const Geom& G, int wx, int wy, int wz, TileSet& s)
{
    s.cx = axis_tiles(wx, G.nx, G.ltx, s.tx);
    s.cy = axis_tiles(wy, G.ny, G.lty, s.ty);
    s.cz = axis_tiles(wz, G.nz, G.ltz, s.tz);
}

// window base of one axis for a point with stencil base b (wrapped) and 1-D weights w:
// w[0] > w[3] exactly when the point lies in the lower half of its cell
template <class T> __device__ __forceinline__ int window_base(int b, int n, const T (&w)[4])
{
    return w[0] > w[3] ? (b == 0 ? n - 1 : b - 1) : b;
}

// the stencil (base b) still lies in the window (base w0) of a periodic axis of length n
__device__ __forceinline__ bool in_window(int b, int w0, int n)
{
    int d = b - w0;
    if (d < 0) d += n;
    return d <= WIN - 4;
}

__device__ __forceinline__ long long tile_id(const Geom& G, int box, int tz, int ty, int tx)
{
    return (((long long)box * G.ntz + tz) * G.nty + ty) * G.ntx + tx;
}

__device__ __forceinline__ int pick(const int (&a)[WIN], int j)
{
    int v = a[0];
#pragma unroll
    for (int q = 1; q < WIN; ++q) v = j == q ? a[q] : v;
    return v;
}

// Tile of slot k of a point (k = (iz cy + iy) cx + ix over its distinct window tiles per
// axis), or -1 past the point's last slot.
__device__ __forceinline__ long long slot_tile(const Geom& G, const TileSet& s, int box, int k)
{
    if (k >= s.cx * s.cy * s.cz) return -1;
    const int ix = k % s.cx, iy = (k / s.cx) % s.cy, iz = k / (s.cx * s.cy);
    return tile_id(G, box, pick(s.tz, iz), pick(s.ty, iy), pick(s.tx, ix));
}

// The (point, slot) kernels run a group of lanes_per_point(maxp) consecutive lanes per point,
// lane k of the group taking slot k: the atomics of one point then run side by side.
int lanes_per_point(int maxp)
{
    int g = 1;
    while (g < maxp) g <<= 1;
    return g;
}

// ---------------------------------------------------------------------------
// 1. records: wrapped base node, one-dimensional weights, force (one thread per
//    point).  err bit 1: box id out of range, bit 2: non-finite input.
//    With psum set (one box), each block also writes the sum of its points'
//    forces (as the records hold them) to psum[blockIdx.x]: the counter-force
//    then needs no pass over the tile lists.
template <class T>
__device__ __forceinline__ void prep_point(const Geom& G, long long i, long long p, const double* __restrict__ pos,
                                           const double* __restrict__ frc, const int* __restrict__ boxid,
                                           PRec<T>* __restrict__ rec, int* __restrict__ err, double (&fs)[3]);

template <class T>
__global__ __launch_bounds__(256) void k_prep(const Geom G, long long n, long long off, const double* __restrict__ pos,
                                              const double* __restrict__ frc, const int* __restrict__ boxid,
                                              PRec<T>* __restrict__ rec, int* __restrict__ err,
                                              double* __restrict__ psum)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    // the list build's grid-barrier counter (err[2]) starts every build at zero
    if (i == 0) err[2] = 0;
    double fs[3] = {0.0, 0.0, 0.0};
    if (i < n) prep_point<T>(G, i, off + i, pos, frc, boxid, rec, err, fs);
    if (!psum) return;
    __shared__ double red[4][3];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = 0; k < 3; ++k) {
        const double v = wave_sum(fs[k]);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int k = threadIdx.x;
        psum[3 * (long long)blockIdx.x + k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    }
}

template <class T>
__device__ __forceinline__ void prep_point(const Geom& G, long long i, long long p, const double* __restrict__ pos,
                                           const double* __restrict__ frc, const int* __restrict__ boxid,
                                           PRec<T>* __restrict__ rec, int* __restrict__ err, double (&fs)[3])
{
    int box = boxid ? boxid[i] : 0;
    if (box < 0 || box >= G.nboxes) {
        atomicOr(err, 1);
        box = 0;
    }
    double R[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    double F[3] = {frc[3 * i], frc[3 * i + 1], frc[3 * i + 2]};
    bool ok = true;
    for (int a = 0; a < 3; ++a) ok = ok && (fabs(R[a]) < 1e300) && (fabs(F[a]) < 1e300);
    if (!ok) {
        atomicOr(err, 2);
        R[0] = R[1] = R[2] = 0.0;
        F[0] = F[1] = F[2] = 0.0;
    }
    const int L[3] = {G.nx, G.ny, G.nz};
    int base[3];
    PRec<T> r;
    for (int a = 0; a < 3; ++a) {
        const double x = wrap_pos(R[a], double(L[a]));
        int b0 = (int)floor(x);
        if (b0 >= L[a]) b0 = L[a] - 1;
        double w[4];
        peskin4(x - b0, w);
        base[a] = b0 == 0 ? L[a] - 1 : b0 - 1;
        T* dst = a == 0 ? r.wx : (a == 1 ? r.wy : r.wz);
        for (int q = 0; q < 4; ++q) dst[q] = T(w[q]);
    }
    r.bx = base[0];
    r.by = base[1];
    r.bz = base[2];
    r.box = box;
    r.f[0] = T(F[0]);
    r.f[1] = T(F[1]);
    r.f[2] = T(F[2]);
    r.pad = T(0);
    rec[p] = r;
    for (int a = 0; a < 3; ++a) fs[a] = double(r.f[a]);
    // skin crossing: the stencil has left the window it was binned with
    const int4 w = G.win[p];
    // (flags read first: after a change of the sets every point is outside its window and
    // both flags are already raised, so no atomics queue up on one address)
    if (!(in_window(r.bx, w.x, G.nx) && in_window(r.by, w.y, G.ny) && in_window(r.bz, w.z, G.nz) && w.w == box)) {
        if (!G.rebox[box]) atomicOr(&G.rebox[box], 1);
        if (!*G.rebin) atomicOr(G.rebin, 1);
    }
}

// 1b-4. The tile lists, rebuilt in one launch (k_rebin) only while the rebuild flag is set.
//    In the usual step (no crossing) every block reads the flag and returns: one kernel
//    boundary per step instead of one per phase.  Otherwise a grid of one block of 256
//    threads per compute unit (at most BIN_GRID; all resident at once) runs four phases
//    separated by grid-wide barriers:
//      1b count the (tile, point) pairs: one group of gp lanes per point (see
//         lanes_per_point), lane k counting the point in the tile of slot k.  Windows are
//         chosen afresh (lane 0 stores them) only for the points of boxes in which a point
//         crossed; the others keep theirs, so what a box computes never depends on crossings
//         in the other boxes of a batch;
//      2  exclusive scan of the per-tile counts into offsets, in chunks of 256 tiles (chunk
//         sums, then each chunk's prefix and scan; integer sums, so the result does not
//         depend on the order); count and cursor are cleared for the next build;
//      3  fill the lists (slot order from atomics), one lane per (point, slot) as in 1b;
//         the per-box crossing flags are cleared (1b, their only reader, has finished);
//      4  sort every tile's list by point index, so that sums run in a fixed order: one
//         thread per entry, its position the number of smaller entries in the same list.
//    A block passes a barrier only when every block has reached it, so whatever a phase
//    reads is complete.  The barrier's wait is bounded: a block that waits too long raises
//    err bit 4 and leaves (the lists then keep a consistent earlier state or miss entries;
//    the step that reads the flags reports the error).
constexpr unsigned BIN_GRID = 256;
constexpr int CHUNK = 256;                 // tiles per scan chunk (threads per block)
constexpr unsigned BARRIER_SPINS = 1u << 20;

// Grid-wide barrier number k (1, 2, ...) of a launch on the counter bar (zeroed by the
// records kernel before every launch).  Returns false if the wait ran out.
__device__ __forceinline__ bool grid_barrier(unsigned* bar, unsigned k, int* err)
{
    __shared__ int ok;
    __syncthreads();   // the block's writes have reached the compute unit's L2 (L1 writes through)
    if (threadIdx.x == 0) {
        // one device-scope release per block: the write-back covers every wave's writes in L2
        __threadfence();
        ok = 1;
        atomicAdd(bar, 1u);
        const unsigned target = k * gridDim.x;
        unsigned n = 0;
        while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++n > BARRIER_SPINS) {
                atomicOr(err, 4);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(8);
        }
        // acquire for the block: the invalidation of L1 and L2 serves every wave's later loads
        __threadfence();
    }
    __syncthreads();
    return ok != 0;
}

// Sum of v over the 256 threads of the block, returned to every thread (fixed order).
__device__ __forceinline__ int block_sum_256(int v, int* sh)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    const int t = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
    return t;
}

// Exclusive scan of v over the 256 threads of the block; total to every thread.
__device__ __forceinline__ int block_exclusive_scan_256(int v, int* sh, int& total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(incl, o, 64);
        if (lane >= o) incl += u;
    }
    if (lane == 63) sh[wave] = incl;
    __syncthreads();
    int pre = 0;
    for (int w = 0; w < wave; ++w) pre += sh[w];
    total = ((sh[0] + sh[1]) + sh[2]) + sh[3];
    __syncthreads();
    return pre + incl - v;
}

template <class T>
__global__ __launch_bounds__(256) void k_rebin(const Geom G, long long npts, int gp, const PRec<T>* __restrict__ rec,
                                               int* __restrict__ count, int* __restrict__ bsum, int* __restrict__ toff,
                                               int* __restrict__ cursor, int* __restrict__ tlist_tmp,
                                               int* __restrict__ tlist, long long max_entries, int* __restrict__ err)
{
    if (!*G.rebin) return;
    __shared__ int sh[4];
    unsigned* bar = reinterpret_cast<unsigned*>(err + 2);
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long gid0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;

    // 1b. count
    for (long long gid = gid0; gid < npts * gp; gid += stride) {
        const long long p = gid / gp;
        const int k = int(gid % gp);
        if (k >= G.maxp) continue;
        const PRec<T> r = rec[p];
        const bool fresh = G.rebox[r.box] != 0;
        const int4 w = fresh ? make_int4(window_base(r.bx, G.nx, r.wx), window_base(r.by, G.ny, r.wy),
                                         window_base(r.bz, G.nz, r.wz), r.box)
                             : G.win[p];
        if (fresh && k == 0) G.win[p] = w;
        TileSet s;
        window_tiles(G, w.x, w.y, w.z, s);
        const long long t = slot_tile(G, s, r.box, k);
        if (t >= 0) atomicAdd(&count[t], 1);
    }
    if (!grid_barrier(bar, 1, err)) return;

    // 2. scan: chunk sums, then each chunk's prefix and exclusive scan
    const long long n = G.ntiles, nch = (n + CHUNK - 1) / CHUNK;
    for (long long c = blockIdx.x; c < nch; c += gridDim.x) {
        const long long i = c * CHUNK + threadIdx.x;
        const int t = block_sum_256(i < n ? count[i] : 0, sh);
        if (threadIdx.x == 0) bsum[c] = t;
    }
    if (!grid_barrier(bar, 2, err)) return;
    for (long long c = blockIdx.x; c < nch; c += gridDim.x) {
        int acc = 0;
        for (long long q = threadIdx.x; q < c; q += CHUNK) acc += bsum[q];
        const int pre = block_sum_256(acc, sh);
        const long long i = c * CHUNK + threadIdx.x;
        const int v = i < n ? count[i] : 0;
        int total;
        const int ex = block_exclusive_scan_256(v, sh, total);
        if (i < n) {
            toff[i] = pre + ex;
            count[i] = 0;
            cursor[i] = 0;
        }
        if (c == nch - 1 && threadIdx.x == 0) toff[n] = pre + total;
    }
    if (!grid_barrier(bar, 3, err)) return;

    // 3. fill
    for (long long b = gid0; b < G.nboxes; b += stride) G.rebox[b] = 0;
    for (long long gid = gid0; gid < npts * gp; gid += stride) {
        const long long p = gid / gp;
        const int k = int(gid % gp);
        const int4 w = G.win[p];
        TileSet s;
        window_tiles(G, w.x, w.y, w.z, s);
        const long long t = slot_tile(G, s, w.w, k);
        if (t < 0) continue;
        // home tile: the one holding the window's centre node (always inside the stencil)
        int cx = w.x + 2, cy = w.y + 2, cz = w.z + 2;
        if (cx >= G.nx) cx -= G.nx;
        if (cy >= G.ny) cy -= G.ny;
        if (cz >= G.nz) cz -= G.nz;
        const bool home = t == tile_id(G, w.w, cz >> G.ltz, cy >> G.lty, cx >> G.ltx);
        const int slot = toff[t] + atomicAdd(&cursor[t], 1);
        tlist_tmp[slot] = int(p << PK_SHIFT) | (home ? PK_HOME : 0) | k;
    }
    if (!grid_barrier(bar, 4, err)) return;

    // 4. sort
    const long long ne = min(max_entries, (long long)toff[G.ntiles]);
    for (long long e = gid0; e < ne; e += stride) {
        const int v = tlist_tmp[e];
        const int p = pk_point(v), k = pk_slot(v);
        const int4 w = G.win[p];
        TileSet s;
        window_tiles(G, w.x, w.y, w.z, s);
        const long long t = slot_tile(G, s, w.w, k);
        const int a = toff[t], b = toff[t + 1];
        int rank = 0;
        for (int j = a; j < b; ++j) rank += tlist_tmp[j] < v ? 1 : 0;
        tlist[a + rank] = v;
    }
}

// ---------------------------------------------------------------------------
// 5. per-box work before a step: the counter-force density -sum F / N and, for
//    FP16 storage, the exponent of the data written by the coming step, chosen
//    from the largest bracket of the last one.  The force sum visits each point
//    once, at its home entry (flagged when the lists are built), striding over
//    the box's own span of the lists in a fixed chunking, so the result does not
//    depend on the other boxes that share the launch or on the order in which
//    the bins were filled.  With one box the records kernel has already summed
//    the forces per block of points (psum, npsum blocks): those sums are added
//    instead, in block order.
// The box's counter-force density from its force sums (four wave sums each) and, for FP16
// storage, the next step's scale exponent from its largest bracket magnitude.
__device__ __forceinline__ void finish_box(const Geom& G, BoxDev& B, const double (&red)[4][3], const float (&redm)[4],
                                           int zero_net, int fp16_exp)
{
    if (zero_net)
        for (int k = 0; k < 3; ++k) B.gc[k] = -(((red[0][k] + red[1][k]) + red[2][k]) + red[3][k]) / double(G.N);
    if (fp16_exp) {
        const float mx = fmaxf(fmaxf(redm[0], redm[1]), fmaxf(redm[2], redm[3]));
        const int e_in = B.e_data;
        int e_out = e_in;
        if (mx > 0.0f && mx < 3.0e38f) {
            const float v = ldexpf(mx, e_in);
            if (v > 32768.0f || v < 4096.0f) e_out = 13 - ilogbf(mx);
        }
        e_out = max(-100, min(120, e_out));
        B.s_in = ldexpf(1.0f, -e_in);
        B.s_out = ldexpf(1.0f, e_out);
        B.e_data = e_out;
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_box_update(const Geom G, const PRec<T>* __restrict__ rec,
                                                    const int* __restrict__ toff, const int* __restrict__ tlist,
                                                    const double* __restrict__ psum, long long npsum,
                                                    const float* __restrict__ tmax, double* __restrict__ part,
                                                    float* __restrict__ pmax, unsigned* __restrict__ ticket,
                                                    BoxDev* __restrict__ boxes, int zero_net, int fp16_exp)
{
    // block (b, c) covers tiles 256 c + thread + 256 C j of box b and the list entries
    // at the same offsets in the box's span (C at most 256: one ticket per block)
    const int b = blockIdx.x, c = blockIdx.y, C = gridDim.y;
    const long long t = (long long)c * blockDim.x + threadIdx.x;
    double s[3] = {0.0, 0.0, 0.0};
    float m = 0.0f;
    if (fp16_exp && G.smax) {
        // one box: the slots the step kernel's tiles raised; cleared for the next step
        for (int u = t; u < SMAX_SLOTS; u += C * blockDim.x) {
            m = fmaxf(m, __uint_as_float(G.smax[u * SMAX_STRIDE]));
            G.smax[u * SMAX_STRIDE] = 0u;
        }
    } else if (fp16_exp) {
        for (long long u = t; u < G.tiles_per_box; u += (long long)C * blockDim.x)
            m = fmaxf(m, tmax[(long long)b * G.tiles_per_box + u]);
    }
    if (zero_net && psum) {
        for (long long u = t; u < npsum; u += (long long)C * blockDim.x)
            for (int k = 0; k < 3; ++k) s[k] += psum[3 * u + k];
    } else if (zero_net && toff) {
        const long long e0 = toff[(long long)b * G.tiles_per_box], e1 = toff[(long long)(b + 1) * G.tiles_per_box];
        const long long S = (long long)C * blockDim.x;
        // the thread's entries e0 + t + S j in increasing j, eight at a time: all list loads,
        // then the forces of the home entries, then the sums in that same order
        for (long long e = e0 + t; e < e1; e += 8 * S) {
            int v[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = e + j * S < e1 ? tlist[e + j * S] : 0;   // 0: not a home entry
            T f[8][3];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const bool h = pk_home(v[j]);
                const PRec<T>& r = rec[h ? pk_point(v[j]) : 0];
                f[j][0] = h ? r.f[0] : T(0);
                f[j][1] = h ? r.f[1] : T(0);
                f[j][2] = h ? r.f[2] : T(0);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j)
                if (pk_home(v[j])) {
                    s[0] += double(f[j][0]);
                    s[1] += double(f[j][1]);
                    s[2] += double(f[j][2]);
                }
        }
    }
    __shared__ double red[4][3];
    __shared__ float redm[4];
    __shared__ int last;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int k = 0; k < 3; ++k) {
        const double v = wave_sum(s[k]);
        if (lane == 0) red[wave][k] = v;
    }
    m = wave_max(m);
    if (lane == 0) redm[wave] = m;
    __syncthreads();
    if (C == 1) {
        // the block is the box's only one: its sums are the box's (the same values the combination
        // below would give: it would add zeros to them), with no partials, fences or tickets
        if (threadIdx.x == 0) finish_box(G, boxes[b], red, redm, zero_net, fp16_exp);
        return;
    }
    if (threadIdx.x == 0) {
        for (int k = 0; k < 3; ++k)
            part[((long long)b * C + c) * 3 + k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
        pmax[(long long)b * C + c] = fmaxf(fmaxf(redm[0], redm[1]), fmaxf(redm[2], redm[3]));
        __threadfence();
        last = (atomicAdd(&ticket[b], 1u) == unsigned(C - 1));
    }
    __syncthreads();
    if (!last) return;
    // the last block of the box combines the C partials in a fixed order
    __threadfence();
    double tot[3] = {0.0, 0.0, 0.0};
    float mx = 0.0f;
    for (int j = threadIdx.x; j < C; j += blockDim.x) {
        for (int k = 0; k < 3; ++k) tot[k] += ((volatile double*)part)[((long long)b * C + j) * 3 + k];
        mx = fmaxf(mx, ((volatile float*)pmax)[(long long)b * C + j]);
    }
    __syncthreads();
    for (int k = 0; k < 3; ++k) {
        const double v = wave_sum(tot[k]);
        if (lane == 0) red[wave][k] = v;
    }
    mx = wave_max(mx);
    if (lane == 0) redm[wave] = mx;
    __syncthreads();
    if (threadIdx.x != 0) return;
    finish_box(G, boxes[b], red, redm, zero_net, fp16_exp);
    ticket[b] = 0u;
}

// ---------------------------------------------------------------------------
// 6. interpolated velocity of each point (sum of its tile partials in a fixed
//    order), optional outputs, and the colloid update with the optional MLP
//    correction to 1/a_L.  A group of ADV_GP lanes per point: lane r of the group
//    sums slots r, r + ADV_GP, ... (all its loads in flight at once), a butterfly
//    over the group adds the lanes' sums (every lane ends with the same bits, as
//    a + b == b + a), and lane 0 of the group finishes the point.
constexpr int ADV_GP = 8;
static_assert((64 / ADV_GP) * ADV_GP >= (1 << PK_BITS), "a group covers every slot a point can have");
struct AdvectArgs {
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
    const unsigned long long* tin;
};

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// The group's sum of point p's partials (every lane of the group returns the same bits).  The
// partials are in the arithmetic type T of the storage (the wave sums of the step kernel);
// the sum is taken in FP64.
template <class T>
__device__ __forceinline__ void group_sum(const Geom& G, const T* __restrict__ partial, long long p, int r,
                                          double (&U)[3])
{
    // the point's partials, one per tile of its window (nt <= maxp <= 64 slots)
    const int4 win = G.win[p];
    const int nt = axis_count(win.x, G.nx, G.ltx) * axis_count(win.y, G.ny, G.lty) * axis_count(win.z, G.nz, G.ltz);
    const T* pp = partial + p * G.maxp * 3;
    double v[64 / ADV_GP][3];
#pragma unroll
    for (int m = 0; m < 64 / ADV_GP; ++m)
#pragma unroll
        for (int c = 0; c < 3; ++c) v[m][c] = r + m * ADV_GP < nt ? double(pp[(r + m * ADV_GP) * 3 + c]) : 0.0;
    U[0] = U[1] = U[2] = 0.0;
#pragma unroll
    for (int m = 0; m < 64 / ADV_GP; ++m)
#pragma unroll
        for (int c = 0; c < 3; ++c) U[c] += v[m][c];
#pragma unroll
    for (int d = 1; d < ADV_GP; d <<= 1)
#pragma unroll
        for (int c = 0; c < 3; ++c) U[c] += __shfl_xor(U[c], d, ADV_GP);
}

__device__ __forceinline__ int point_box(const Geom& G, const AdvectArgs& A, long long i)
{
    const int box = A.boxid ? A.boxid[i] : 0;
    return (box < 0 || box >= G.nboxes) ? 0 : box;
}

// Outputs and the move of point i (set-local; p = A.off + i) with interpolated velocity U;
// y: the network's output for the point (used only with A.mlp).
__device__ __forceinline__ void finish_point(const Geom& G, const AdvectArgs& A, const BoxDev* __restrict__ boxes,
                                             long long i, long long p, const double (&U)[3], float y)
{
    for (int c = 0; c < 3; ++c) {
        if (A.vel_out) A.vel_out[3 * i + c] = U[c];
        if (A.vel_sum) A.vel_sum[3 * i + c] += U[c];
    }
    if (!A.advect) return;
    const int box = point_box(G, A, i);
    double inv_aL = A.inv_aL;
    if (A.mlp) inv_aL += double(A.out_scale) * double(y);
    const double R[3] = {A.pos[3 * i], A.pos[3 * i + 1], A.pos[3 * i + 2]};
    const double L[3] = {double(G.nx), double(G.ny), double(G.nz)};
    const double mob = (A.inv_a - inv_aL) * boxes[box].inv6pe;
    double zeta[3] = {0.0, 0.0, 0.0};
    if (A.tin) {
        // Appendix B: extra Brownian displacement, variance kT/(3 pi eta)(1/a - 1/a_L) per step
        const Philox4 q = particle_draw(uint32_t(p), *A.tin, G.seed_lo, G.seed_hi);
        double z[4];
        box_muller<double>(q.v[0], q.v[1], z[0], z[1]);
        box_muller<double>(q.v[2], q.v[3], z[2], z[3]);
        const double amp = sqrt(boxes[box].pn * fmax(A.inv_a - inv_aL, 0.0));
        for (int a = 0; a < 3; ++a) zeta[a] = amp * z[a];
    }
    for (int a = 0; a < 3; ++a)
        A.pos[3 * i + a] = wrap_pos(R[a] + (U[a] + zeta[a]) + A.frc[3 * i + a] * mob, L[a]);
}

// Without the MLP: one group per point, lane 0 of the group finishes it.
template <class T>
__global__ __launch_bounds__(256) void k_advect(const Geom G, const AdvectArgs A, const BoxDev* __restrict__ boxes,
                                                const T* __restrict__ partial)
{
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long i = gid / ADV_GP;
    const int r = int(gid % ADV_GP);
    if (i >= A.n) return;   // whole groups: a group is 8 aligned lanes of one wave
    double U[3];
    group_sum(G, partial, A.off + i, r, U);
    if (r == 0) finish_point(G, A, boxes, i, A.off + i, U, 0.0f);
}

// With the MLP correction to 1/a_L (4 -> 64 tanh -> 64 tanh -> 1, bf16 weights staged in LDS
// as FP32, FP32 products and sums).  A block of MLP_WAVES waves takes 64 points: the
// interpolation partials are summed first (groups of ADV_GP lanes per point, as in k_advect);
// wave w evaluates the first-layer units j = 16 w .. 16 w + 15 of every point (one point per
// lane) into LDS; the second layer is a 64 x 64 by 64 x 64 product on the matrix cores (FP32
// MFMA, 32 x 32 x 2 steps): wave w takes the 32 units 32 (w & 1) .. and the 32 points
// 32 (w >> 1) .. of one output tile, applies tanh and the output weights to its 16 values per
// lane, and the two halves of the units are added (lanes l and l ^ 32, then the two waves of a
// point half in order).  tanh(s) = 1 - 2 / (exp(2 s) + 1) with the hardware exponential and
// reciprocal (absolute error ~1e-7).
constexpr int MLP_H = 64;
constexpr int MLP_WAVES = 4;
constexpr int MLP_UNITS = MLP_H / MLP_WAVES;
constexpr int MLP_BLOCK = 64 * MLP_WAVES;

__device__ __forceinline__ float tanh_fast(float s)
{
    const float e = __builtin_amdgcn_exp2f(s * 2.8853900817779268f);   // exp(2 s)
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

typedef float mfma_acc16 __attribute__((ext_vector_type(16)));

template <class T>
__global__ __launch_bounds__(MLP_BLOCK) void k_advect_mlp(const Geom G, const AdvectArgs A,
                                                          const BoxDev* __restrict__ boxes,
                                                          const T* __restrict__ partial)
{
    __shared__ float4 W1[MLP_H];                         // rows of W1 (4 inputs)
    __shared__ float b1[MLP_H], b2[MLP_H], W3[MLP_H];
    __shared__ float W2T[MLP_H][MLP_H + 1];              // W2 transposed: [input k][unit] (padded row)
    __shared__ float h1[MLP_H][64];                      // [unit][point of the block]
    __shared__ double Us[64][3];
    __shared__ float ys[2][64];
    __shared__ float b3;
    // lbml layout: W1[64][4], b1[64], W2[64][64], b2[64], W3[1][64], b3[1]; the block's share of
    // the weights is loaded first and staged after the interpolation sums below, so that the two
    // sets of loads are in flight together
    constexpr int WPT = (LBML_NPARAM_DEV + MLP_BLOCK - 1) / MLP_BLOCK;
    uint16_t wraw[WPT];
#pragma unroll
    for (int j = 0; j < WPT; ++j) {
        const int k = int(threadIdx.x) + j * MLP_BLOCK;
        wraw[j] = k < LBML_NPARAM_DEV ? A.mlp[k] : uint16_t(0);
    }
    const long long base = (long long)blockIdx.x * 64;
    // interpolated velocity of the block's points: ADV_GP lanes per point, MLP_BLOCK / ADV_GP at a time
    for (int pl0 = 0; pl0 < 64; pl0 += MLP_BLOCK / ADV_GP) {
        const int pl = pl0 + int(threadIdx.x) / ADV_GP, r = int(threadIdx.x) % ADV_GP;
        const long long i = min(base + pl, A.n - 1);
        double U[3];
        group_sum(G, partial, A.off + i, r, U);
        if (r == 0) {
            Us[pl][0] = U[0];
            Us[pl][1] = U[1];
            Us[pl][2] = U[2];
        }
    }
#pragma unroll
    for (int j = 0; j < WPT; ++j) {
        const int k = int(threadIdx.x) + j * MLP_BLOCK;
        if (k >= LBML_NPARAM_DEV) continue;
        const float v = bf16_to_f32(wraw[j]);
        if (k < 256) reinterpret_cast<float*>(W1)[k] = v;
        else if (k < 320) b1[k - 256] = v;
        else if (k < 4416) W2T[(k - 320) % MLP_H][(k - 320) / MLP_H] = v;
        else if (k < 4480) b2[k - 4416] = v;
        else if (k < 4544) W3[k - 4480] = v;
        else b3 = v;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
    const bool live = base + lane < A.n;
    const long long i = live ? base + lane : A.n - 1;   // lanes past the end repeat the last point
    // inputs: fractional offsets of the (wrapped) position and the box's tau
    float xin[4];
    {
        const double L[3] = {double(G.nx), double(G.ny), double(G.nz)};
        for (int a = 0; a < 3; ++a) {
            const double R = wrap_pos(A.pos[3 * i + a], L[a]);
            xin[a] = (float(R - floor(R)) - A.in_shift[a]) * A.in_scale[a];
        }
        xin[3] = (float(boxes[point_box(G, A, i)].tau) - A.in_shift[3]) * A.in_scale[3];
    }
#pragma unroll
    for (int q = 0; q < MLP_UNITS; ++q) {
        const int j = wave * MLP_UNITS + q;
        const float4 w = W1[j];
        float s = b1[j];
        s = fmaf(w.x, xin[0], s);
        s = fmaf(w.y, xin[1], s);
        s = fmaf(w.z, xin[2], s);
        s = fmaf(w.w, xin[3], s);
        h1[j][lane] = tanh_fast(s);
    }
    __syncthreads();
    // second layer, one 32 x 32 tile per wave: A = W2 rows (units), B = first-layer values
    // (columns = points); step ks takes inputs 2 ks (lanes 0-31) and 2 ks + 1 (lanes 32-63)
    const int uh = wave & 1, ph = wave >> 1, c32 = lane & 31, kh = lane >> 5;
    mfma_acc16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
    for (int ks = 0; ks < MLP_H / 2; ++ks) {
        const int k = 2 * ks + kh;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(W2T[k][32 * uh + c32], h1[k][32 * ph + c32], acc, 0, 0, 0);
    }
    // lane: point 32 ph + c32, units 32 uh + 8 (r / 4) + 4 kh + r % 4 of the tile
    float y = 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int u = 32 * uh + 8 * (r >> 2) + 4 * kh + (r & 3);
        y = fmaf(W3[u], tanh_fast(acc[r] + b2[u]), y);
    }
    y += __shfl_xor(y, 32);
    if (kh == 0) ys[uh][32 * ph + c32] = y;
    __syncthreads();
    if (wave == 0 && live) {
        const double U[3] = {Us[lane][0], Us[lane][1], Us[lane][2]};
        finish_point(G, A, boxes, i, A.off + i, U, (ys[0][lane] + ys[1][lane]) + b3);
    }
}

// ---------------------------------------------------------------------------
// 7. interpolation at arbitrary points: one wave per point, one lane per
//    stencil node; each lane rebuilds u at its node from the stored
//    populations and the binned forces.
template <int ST>
__global__ __launch_bounds__(256) void k_interp_points(const Geom G, long long n, const double* __restrict__ pos,
                                                       const int* __restrict__ boxid, double* __restrict__ out,
                                                       const typename StoreT<ST>::S* __restrict__ src,
                                                       const BoxDev* __restrict__ boxes, const int* __restrict__ toff,
                                                       const int* __restrict__ tlist,
                                                       const PRec<typename StoreT<ST>::T>* __restrict__ rec)
{
    using T = typename StoreT<ST>::T;
    const int lane = threadIdx.x & 63;
    const long long q = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (q >= n) return;
    int box = boxid ? boxid[q] : 0;
    if (box < 0 || box >= G.nboxes) box = 0;
    const int d[3] = {lane & 3, (lane >> 2) & 3, lane >> 4};
    const int L[3] = {G.nx, G.ny, G.nz};
    int node[3];
    double wt = 1.0;
    for (int a = 0; a < 3; ++a) {
        const double x = wrap_pos(pos[3 * q + a], double(L[a]));
        int b0 = (int)floor(x);
        if (b0 >= L[a]) b0 = L[a] - 1;
        double w[4];
        peskin4(x - b0, w);
        int nd = b0 - 1 + d[a];
        if (nd < 0) nd += L[a];
        if (nd >= L[a]) nd -= L[a];
        node[a] = nd;
        wt *= w[d[a]];
    }
    const int x = node[0], y = node[1], z = node[2];
    const int xm = x == 0 ? G.nx - 1 : x - 1, xp = x + 1 == G.nx ? 0 : x + 1;
    const int ym = y == 0 ? G.ny - 1 : y - 1, yp = y + 1 == G.ny ? 0 : y + 1;
    const int zm = z == 0 ? G.nz - 1 : z - 1, zp = z + 1 == G.nz ? 0 : z + 1;
    const auto* sb = src + (long long)box * G.sbox;
    const BoxDev& B = boxes[box];
    T f[NQ];
    pull_node<ST, false, A_G64>(sb, G.rb, G.kp, 0u, G.ny, x, y, z, xm, xp, ym, yp, zm, zp,
                         f);
    T drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const T v = f[i];
        drho += v;
        if (cvel(i, 0) != 0) jx += cvel(i, 0) > 0 ? v : -v;
        if (cvel(i, 1) != 0) jy += cvel(i, 1) > 0 ? v : -v;
        if (cvel(i, 2) != 0) jz += cvel(i, 2) > 0 ? v : -v;
    }
    if constexpr (ST == ST_FP16) {
        const T s = T(ldexpf(1.0f, -B.e_data));
        drho *= s;
        jx *= s;
        jy *= s;
        jz *= s;
    }
    T gx = T(B.gc[0]), gy = T(B.gc[1]), gz = T(B.gc[2]);
    if (toff) {
        const long long t = tile_id(G, box, z >> G.ltz, y >> G.lty, x >> G.ltx);
        for (int k = toff[t]; k < toff[t + 1]; ++k) {
            const PRec<T>& r = rec[pk_point(tlist[k])];
            const T w = stencil_w<T>(x, r.bx, G.nx, r.wx) * stencil_w<T>(y, r.by, G.ny, r.wy) *
                        stencil_w<T>(z, r.bz, G.nz, r.wz);
            gx += r.f[0] * w;
            gy += r.f[1] * w;
            gz += r.f[2] * w;
        }
    }
    const T rho = T(G.rho0) + drho;
    const T ir = T(1) / rho;
    const double u[3] = {double((jx + T(0.5) * gx) * ir), double((jy + T(0.5) * gy) * ir),
                         double((jz + T(0.5) * gz) * ir)};
    for (int c = 0; c < 3; ++c) {
        const double s = wave_sum(wt * u[c]);
        if (lane == 0) out[3 * q + c] = s;
    }
}

// ---------------------------------------------------------------------------
// 8. diagnostics: per-box reduction of the per-tile partials in tile order
__global__ __launch_bounds__(256) void k_diag_reduce(const Geom G, const double* __restrict__ part,
                                                     double* __restrict__ out)
{
    const int b = blockIdx.x;
    __shared__ double red[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c = 0; c < LBD_N; ++c) {
        double a = 0.0;
        for (long long t = threadIdx.x; t < G.tiles_per_box; t += blockDim.x) {
            const double v = part[((long long)b * G.tiles_per_box + t) * LBD_N + c];
            a = c == 10 ? fmax(a, v) : a + v;
        }
        a = c == 10 ? wave_max(a) : wave_sum(a);
        if (lane == 0) red[wave] = a;
        __syncthreads();
        if (threadIdx.x == 0)
            out[(long long)b * LBD_N + c] =
                c == 10 ? fmax(fmax(red[0], red[1]), fmax(red[2], red[3])) : ((red[0] + red[1]) + red[2]) + red[3];
        __syncthreads();
    }
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, long long n, uint32_t v)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// launchers

static unsigned nblk(long long n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_fill_u32(void* p, long long n, uint32_t v, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_u32, dim3(nblk(n, 256)), dim3(256), 0, s, (uint32_t*)p, n, v);
}

long long prep_blocks(long long n) { return n > 0 ? nblk(n, 256) : 0; }

void launch_prep(int storage, const Geom& G, long long n, long long off, const double* pos, const double* frc,
                 const int* boxid, void* rec, int* err, double* psum, hipStream_t s)
{
    if (n <= 0) return;
    if (storage == ST_FP64)
        hipLaunchKernelGGL(k_prep<double>, dim3(nblk(n, 256)), dim3(256), 0, s, G, n, off, pos, frc, boxid,
                           (PRec<double>*)rec, err, psum);
    else
        hipLaunchKernelGGL(k_prep<float>, dim3(nblk(n, 256)), dim3(256), 0, s, G, n, off, pos, frc, boxid,
                           (PRec<float>*)rec, err, psum);
}

long long scan_blocks(long long ntiles) { return (ntiles + CHUNK - 1) / CHUNK; }

// Blocks of the list build: one per compute unit of the current device, at most BIN_GRID,
// so that the grid is resident at once even on a partition of the GPU.
static unsigned rebin_grid()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 32;
    return std::min<unsigned>(BIN_GRID, unsigned(cus));
}

// Steps 1b-4 over all npts points, after the records of every set are written
// (any set may raise the rebuild flag; the records kernel zeroed the barrier counter).
void launch_bins(int storage, const Geom& G, long long npts, const void* rec, int* count, int* bsum, int* toff,
                 int* cursor, int* tlist, int* tlist_tmp, int* err, hipStream_t s)
{
    if (npts <= 0) return;
    const int gp = lanes_per_point(G.maxp);
    const long long max_entries = npts * G.maxp;
    const unsigned nb = rebin_grid();
    if (storage == ST_FP64)
        hipLaunchKernelGGL(k_rebin<double>, dim3(nb), dim3(256), 0, s, G, npts, gp, (const PRec<double>*)rec, count,
                           bsum, toff, cursor, tlist_tmp, tlist, max_entries, err);
    else
        hipLaunchKernelGGL(k_rebin<float>, dim3(nb), dim3(256), 0, s, G, npts, gp, (const PRec<float>*)rec, count,
                           bsum, toff, cursor, tlist_tmp, tlist, max_entries, err);
}

void launch_box_update(int storage, const Geom& G, const void* rec, const int* toff, const int* tlist,
                       const double* psum, long long npsum, const float* tmax, double* part, float* pmax,
                       unsigned* ticket, BoxDev* boxes, int zero_net, int fp16_exp, hipStream_t s)
{
    // one box whose sums come from the records kernel and whose FP16 maximum from the slots:
    // little to read, one block
    const bool small = G.nboxes == 1 && (psum || !zero_net) && (G.smax || !fp16_exp);
    const dim3 grid(G.nboxes, small ? 1 : G.bchunks);
    if (storage == ST_FP64)
        hipLaunchKernelGGL(k_box_update<double>, grid, dim3(256), 0, s, G, (const PRec<double>*)rec, toff, tlist, psum,
                           npsum, tmax, part, pmax, ticket, boxes, zero_net, fp16_exp);
    else
        hipLaunchKernelGGL(k_box_update<float>, grid, dim3(256), 0, s, G, (const PRec<float>*)rec, toff, tlist, psum,
                           npsum, tmax, part, pmax, ticket, boxes, zero_net, fp16_exp);
}


void launch_advect(int storage, const Geom& G, const AdvectLaunch& a, const BoxDev* boxes, void* partial,
                   hipStream_t s)
{
    if (a.n <= 0) return;
    AdvectArgs A;
    A.n = a.n;
    A.off = a.off;
    A.frc = a.frc;
    A.pos = a.pos;
    A.vel_out = a.vel_out;
    A.vel_sum = a.vel_sum;
    A.boxid = a.boxid;
    A.inv_a = a.inv_a;
    A.inv_aL = a.inv_aL;
    A.mlp = a.mlp;
    for (int k = 0; k < 4; ++k) {
        A.in_shift[k] = a.in_shift[k];
        A.in_scale[k] = a.in_scale[k];
    }
    A.out_scale = a.out_scale;
    A.advect = a.advect;
    A.tin = a.tin;
    const unsigned nb = nblk(a.n * ADV_GP, 256);
    const unsigned nbm = nblk(a.n, 64);   // with the network: 64 points per block
    if (storage == ST_FP64) {
        if (A.mlp)
            hipLaunchKernelGGL(k_advect_mlp<double>, dim3(nbm), dim3(MLP_BLOCK), 0, s, G, A, boxes, (const double*)partial);
        else
            hipLaunchKernelGGL(k_advect<double>, dim3(nb), dim3(256), 0, s, G, A, boxes, (const double*)partial);
    } else {
        if (A.mlp)
            hipLaunchKernelGGL(k_advect_mlp<float>, dim3(nbm), dim3(MLP_BLOCK), 0, s, G, A, boxes, (const float*)partial);
        else
            hipLaunchKernelGGL(k_advect<float>, dim3(nb), dim3(256), 0, s, G, A, boxes, (const float*)partial);
    }
}

void launch_interp_points(int storage, const Geom& G, long long n, const double* pos, const int* boxid, double* out,
                          const void* src, const BoxDev* boxes, const int* toff, const int* tlist, const void* rec,
                          hipStream_t s)
{
    if (n <= 0) return;
    const unsigned nb = nblk(n, 4);
    switch (storage) {
    case ST_FP64:
        hipLaunchKernelGGL(k_interp_points<ST_FP64>, dim3(nb), dim3(256), 0, s, G, n, pos, boxid, out,
                           (const double*)src, boxes, toff, tlist, (const PRec<double>*)rec);
        break;
    case ST_FP32:
        hipLaunchKernelGGL(k_interp_points<ST_FP32>, dim3(nb), dim3(256), 0, s, G, n, pos, boxid, out,
                           (const float*)src, boxes, toff, tlist, (const PRec<float>*)rec);
        break;
    case ST_FP16:
        hipLaunchKernelGGL(k_interp_points<ST_FP16>, dim3(nb), dim3(256), 0, s, G, n, pos, boxid, out,
                           (const _Float16*)src, boxes, toff, tlist, (const PRec<float>*)rec);
        break;
    case ST_MOM32:
        hipLaunchKernelGGL(k_interp_points<ST_MOM32>, dim3(nb), dim3(256), 0, s, G, n, pos, boxid, out,
                           (const float*)src, boxes, toff, tlist, (const PRec<float>*)rec);
        break;
    }
}

void launch_diag_reduce(const Geom& G, const double* part, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_diag_reduce, dim3(G.nboxes), dim3(256), 0, s, G, part, out);
}

}  // namespace lbm

// Device-side definitions shared by the liblbm kernels (gfx950).
//
// Velocity set: D3Q19 (the DdQn quadrature of Sec. II with the standard
// 19-velocity set), listed here as rest, the six faces and the twelve edges,
// each followed by its opposite.  Weights 1/3, 1/18, 1/36; c_s^2 = 1/3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int NQ = 19;
constexpr int BLOCK = 256;  // threads per block of the lattice kernels (4 wave64s)

__host__ __device__ constexpr int cvel(int i, int a)
{
    constexpr int t[NQ][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
                              {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1},
                              {-1, 0, 1}, {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    return t[i][a];
}

__host__ __device__ constexpr double wgt(int i) { return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }

// the kernels rely on velocities 2k+1 and 2k+2 being opposite
constexpr bool opposite_pairs()
{
    for (int i = 1; i < NQ; i += 2)
        for (int a = 0; a < 3; ++a)
            if (cvel(i + 1, a) != -cvel(i, a)) return false;
    return true;
}
static_assert(opposite_pairs(), "velocity table must list opposite pairs");

enum Storage { ST_FP64 = 0, ST_FP32 = 1, ST_FP16 = 2, ST_MOM32 = 3 };

template <int ST> struct StoreT;
template <> struct StoreT<ST_FP64> { using S = double; using T = double; };
template <> struct StoreT<ST_FP32> { using S = float; using T = float; };
template <> struct StoreT<ST_FP16> { using S = _Float16; using T = float; };
template <> struct StoreT<ST_MOM32> { using S = float; using T = float; };

// Moment storage: with the ghosts projected out, the post-collision state of a
// node is fixed by 10 numbers (Eq. fiexp); they are stored as the pieces of
// the bracket f*_i / w_i = r0 + c_i.a + sum_a c_ia^2 b_aa + sum_{a<b} c_ia c_ib b_ab:
//   r0 = drho - (3/2) tr B,  a = 3 A,  b_aa = (9/2) B_aa,  b_ab = 9 B_ab.
enum MomPlane { MP_R0 = 0, MP_AX, MP_AY, MP_AZ, MP_BXX, MP_BYY, MP_BZZ, MP_BXY, MP_BXZ, MP_BYZ, MP_N };

__host__ __device__ constexpr int planes_of(int st) { return st == ST_MOM32 ? MP_N : NQ; }

// Entries of the per-tile point lists: point index (bits 7..30), a flag marking
// the point's home tile (bit 6: the tile holding the centre node of its binning
// window, one per point) and the index of this tile among the tiles of the
// point's window (bits 0..5).  Within one tile's list the order is the order of
// the point indices.
constexpr int PK_BITS = 6;
constexpr int PK_HOME = 1 << PK_BITS;
constexpr int PK_SHIFT = PK_BITS + 1;
__host__ __device__ constexpr int pk_point(int e) { return e >> PK_SHIFT; }
__host__ __device__ constexpr int pk_slot(int e) { return e & ((1 << PK_BITS) - 1); }
__host__ __device__ constexpr bool pk_home(int e) { return (e & PK_HOME) != 0; }

// Per-point record rebuilt before every step that needs it: base node of the
// 4-wide stencil (floor(R) - 1, wrapped), the three sets of one-dimensional
// kernel weights, and the force, in the arithmetic type of the storage mode.
template <class T> struct alignas(16) PRec {
    int bx, by, bz, box;
    T wx[4], wy[4], wz[4];
    T f[3];
    T pad;
};

// FP16 maxima of a one-box lattice: slots and their spacing (one 128-byte line each)
constexpr int SMAX_SLOTS = 256;
constexpr int SMAX_STRIDE = 32;

// Per-box parameters read by the step kernels.
struct alignas(16) BoxDev {
    double tau;
    double omega;      // 1 / (tau + 1/2)
    double gc[3];      // uniform counter-force density (zero unless requested)
    double tau_b;      // bulk relaxation time (general collision)
    double omega_b;    // 1 / (tau_b + 1/2)
    double kappa_g;    // ghost moments are multiplied by this per step (0: projected out)
    double nz_b;       // thermal noise: sqrt(mu (1 - gamma^2)) of the bulk mode (mu = kT / cs^2)
    double nz_s;       // ... of the shear modes
    double nz_g;       // ... of the ghost modes
    double pn;         // particle noise: variance kT / (3 pi eta) per unit of 1/a - 1/a_L
    double inv6pe;     // 1 / (6 pi eta), eta = rho0 tau / 3: the Stokes mobility of the colloid update
    float s_in;        // FP16: dequantise multiplier 2^-e of the stored data
    float s_out;       // FP16: quantise multiplier 2^e of the data written this step
    int e_data;        // FP16: exponent of the data currently stored
    unsigned spare;
};

// Geometry of the lattice and its tiles (all boxes share it).
struct Geom {
    int nx, ny, nz, nboxes;
    int tx, ty, tz;       // tile extent per axis (tx * ty * tz == BLOCK), powers of two
    int ltx, lty, ltz;    // their base-2 logarithms
    int ntx, nty, ntz;    // tiles per axis
    unsigned mtx, mty, mtz;   // for n < 2^31: n / nt = (n * m) >> s (multipliers and shifts set
    int stx, sty, stz;        // on the host, so the step kernel divides without a reciprocal)
    int maxp;             // most tiles met by one point's binning window (5 nodes per axis)
    int bchunks;          // blocks per box of the per-box force / maximum reductions
    int tpb;              // tiles per block of the step kernel
    int order;            // 0: blocks renumbered into contiguous runs per XCD; 1: launch order;
                          // 2: launch order of tile rows, the runs of one tile row on one XCD
    int lgrp;             // order 2: base-2 logarithm of the runs per tile row
    int pairs;            // FP16 step: two adjacent x nodes per lane (nx even)
    int* nf;              // per box, sticky: non-finite value or FP16 overflow seen by a step
    int* rebin;           // set when a point's stencil has left its binning window (tile lists stale)
    int* rebox;           // per box: a point of the box left its window (its windows are chosen again)
    int4* win;            // per point: window base (x, y, z) and box the tile lists were built with
    unsigned* smax;       // FP16, one box: the box's largest bracket as float bits, spread over
                          // SMAX_SLOTS slots a cache line apart (tile t updates slot t % SMAX_SLOTS);
                          // NULL: per-tile maxima instead
    int coll;             // 1: general collision (bulk rate, ghost moments kept); 2: with thermal noise
    float one;            // 1.0: a multiplier the compiler cannot fold, so that the sum of two FP16
                          // values stays one mixed-precision multiply-add (v_fma_mix)
    unsigned seed_lo, seed_hi;   // key of the noise generator
    long long N;          // nodes per box
    long long rb;         // elements between consecutive rows of one plane (see pop_index)
    long long kp;         // elements between consecutive planes of one row
    long long sbox;       // elements between boxes
    long long tiles_per_box;
    long long ntiles;
    double rho0;
};

// Blocks are dealt round-robin to the 8 XCDs; renumber them so that each XCD
// works through a contiguous run of tiles (neighbouring tiles share cache
// lines of the x-shifted pulls and are then served by the same L2).
// n / d for n < 2^31 with the multiplier m = ceil(2^s / d), s = 31 + ceil(log2 d), that the
// host computes: the product's error stays below one part in 2^31 of the quotient's unit.
__device__ __forceinline__ unsigned div_magic(unsigned n, unsigned m, int s)
{
    return unsigned(((unsigned long long)n * m) >> s);
}

__device__ __forceinline__ int xcd_tile(int b, int nblocks)
{
    const int q = nblocks >> 3, r = nblocks & 7;
    const int xcd = b & 7, j = b >> 3;
    return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + j;
}

// Run of block b when the 2^lg runs of each tile row go to one XCD back to back while
// the tile rows themselves still advance in launch order across the XCDs: the k-th
// block the dispatcher sends to XCD j (b = 8k + j) takes run (k mod 2^lg) of tile row
// 8 (k div 2^lg) + j.  The x-neighbours a tile's pull reads at its edges are then in
// the L2 of the XCD that reads them.  Blocks past the last whole group of 8 tile rows
// keep their own run (the map is a bijection on [0, nblocks)).
__device__ __forceinline__ int row_group_run(int b, int nblocks, int lg)
{
    const int whole = (nblocks >> (lg + 3)) << (lg + 3);
    if (b >= whole) return b;
    const int k = b >> 3, j = b & 7;
    return ((((k >> lg) << 3) + j) << lg) + (k & ((1 << lg) - 1));
}

// a = first term or a + x: with the flag a compile-time constant after unrolling, a sum over a
// fixed set of terms starts at its first term instead of adding it to zero
template <class T>
__device__ __forceinline__ void acc_first(T& a, bool& set, T x)
{
    a = set ? a + x : x;
    set = true;
}

// Post-collision brackets f*_i / w_i of the opposite pair (i, i + 1) from the ten pieces of
// Eq. fiexp (order of MomPlane): the even part r0 + sum c_ia^2 b_aa + sum c_ia c_ib b_ab is
// shared, the odd part c_i.a changes sign.
template <class T>
__device__ __forceinline__ void rebuild_pair(const T (&p)[MP_N], int i, T& plus, T& minus)
{
    const int cx = cvel(i, 0), cy = cvel(i, 1), cz = cvel(i, 2);
    T ev = p[MP_R0], od = 0;
    bool s_od = false;
    if (cx != 0) { acc_first(od, s_od, cx > 0 ? p[MP_AX] : -p[MP_AX]); ev += p[MP_BXX]; }
    if (cy != 0) { acc_first(od, s_od, cy > 0 ? p[MP_AY] : -p[MP_AY]); ev += p[MP_BYY]; }
    if (cz != 0) { acc_first(od, s_od, cz > 0 ? p[MP_AZ] : -p[MP_AZ]); ev += p[MP_BZZ]; }
    if (cx * cy != 0) ev += cx * cy > 0 ? p[MP_BXY] : -p[MP_BXY];
    if (cx * cz != 0) ev += cx * cz > 0 ? p[MP_BXZ] : -p[MP_BXZ];
    if (cy * cz != 0) ev += cy * cz > 0 ? p[MP_BYZ] : -p[MP_BYZ];
    plus = ev + od;
    minus = ev - od;
}

// One-dimensional weight of a stencil whose first node is `base` at node
// coordinate `x` on a periodic axis of length n.
template <class T>
__device__ __forceinline__ T stencil_w(int x, int base, int n, const T (&w)[4])
{
    int d = x - base;
    if (d < 0) d += n;
    return d == 0 ? w[0] : d == 1 ? w[1] : d == 2 ? w[2] : d == 3 ? w[3] : T(0);
}

// Cross-lane moves within a wave64 (DPP).  Lanes whose source is outside the
// pattern, or whose row is masked off, receive 0.
template <int CTRL, int ROW, int BANK, bool BC>
__device__ __forceinline__ float dpp(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW, BANK, BC));
}

template <int CTRL, int ROW, int BANK, bool BC>
__device__ __forceinline__ double dpp(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW, BANK, BC);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW, BANK, BC);
    return __builtin_bit_cast(double, (long long)(unsigned)lo | ((long long)hi << 32));
}

__device__ __forceinline__ float lane63(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

__device__ __forceinline__ double lane63(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)b, 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __builtin_bit_cast(double, (long long)(unsigned)lo | ((long long)hi << 32));
}

// Sum over the 64 lanes (all lanes must be active), returned to every lane.
// Fixed tree: shifts by 1, 2, 4, 8 within each 16-lane row, then row 0 -> 1
// and row 2 -> 3 (row_bcast:15), then rows 0-1 -> 2-3 (row_bcast:31); lane 63
// ends with the total.
template <class T>
__device__ __forceinline__ T wave_sum(T v)
{
    v += dpp<0x111, 0xf, 0xf, true>(v);
    v += dpp<0x112, 0xf, 0xf, true>(v);
    v += dpp<0x114, 0xf, 0xf, true>(v);
    v += dpp<0x118, 0xf, 0xf, true>(v);
    v += dpp<0x142, 0xa, 0xf, false>(v);
    v += dpp<0x143, 0xc, 0xf, false>(v);
    return lane63(v);
}

// Maximum over the 64 lanes of non-negative values (masked lanes read 0).
template <class T>
__device__ __forceinline__ T wave_max(T v)
{
    v = fmax(v, dpp<0x111, 0xf, 0xf, true>(v));
    v = fmax(v, dpp<0x112, 0xf, 0xf, true>(v));
    v = fmax(v, dpp<0x114, 0xf, 0xf, true>(v));
    v = fmax(v, dpp<0x118, 0xf, 0xf, true>(v));
    v = fmax(v, dpp<0x142, 0xa, 0xf, false>(v));
    v = fmax(v, dpp<0x143, 0xc, 0xf, false>(v));
    return lane63(v);
}

// Maximum over the 64 lanes of non-negative floats (or NaN), returned to every lane: such
// floats order as their bit patterns, so the tree of wave_max runs on integers (one DPP
// integer max per level; fmax would first quiet each operand).
__device__ __forceinline__ float wave_max_nonneg(float v)
{
    unsigned u = __float_as_uint(v);
    u = max(u, unsigned(__builtin_amdgcn_update_dpp(0, int(u), 0x111, 0xf, 0xf, true)));
    u = max(u, unsigned(__builtin_amdgcn_update_dpp(0, int(u), 0x112, 0xf, 0xf, true)));
    u = max(u, unsigned(__builtin_amdgcn_update_dpp(0, int(u), 0x114, 0xf, 0xf, true)));
    u = max(u, unsigned(__builtin_amdgcn_update_dpp(0, int(u), 0x118, 0xf, 0xf, true)));
    u = max(u, unsigned(__builtin_amdgcn_update_dpp(0, int(u), 0x142, 0xa, 0xf, false)));
    u = max(u, unsigned(__builtin_amdgcn_update_dpp(0, int(u), 0x143, 0xc, 0xf, false)));
    return __uint_as_float(unsigned(__builtin_amdgcn_readlane(int(u), 63)));
}

// Peskin's 4-point kernel at the four nodes floor(r)-1 .. floor(r)+2 for a
// point at fractional offset f = r - floor(r) in [0, 1): Eq. deltadef at
// distances 1+f, f, 1-f, 2-f, which share the root q = sqrt(1 + 4f - 4f^2).
__device__ __forceinline__ void peskin4(double f, double (&w)[4])
{
    const double q = sqrt(1.0 + 4.0 * f - 4.0 * f * f);
    w[0] = (3.0 - 2.0 * f - q) * 0.125;
    w[1] = (3.0 - 2.0 * f + q) * 0.125;
    w[2] = (1.0 + 2.0 * f + q) * 0.125;
    w[3] = (1.0 + 2.0 * f - q) * 0.125;
}

// Raw buffer access: a wave-uniform descriptor (scalar registers) over a row
// block, a plane or a whole box, and a 32-bit byte offset per lane.  The descriptor's
// record count is the size of that range, so an offset past it reads 0 / drops
// the store instead of touching other memory.  Dword 3 is the gfx9-family
// value; aux bit 1 marks the access non-temporal.
using rsrc_t = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ rsrc_t plane_rsrc(const void* base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

template <class S, int AUX>
__device__ __forceinline__ S bload(rsrc_t r, unsigned off, unsigned soff = 0)
{
    if constexpr (sizeof(S) == 8)
        return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, AUX));
    else if constexpr (sizeof(S) == 4)
        return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, AUX));
    else
        return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b16(r, off, soff, AUX));
}

template <class S, int AUX>
__device__ __forceinline__ void bstore(S v, rsrc_t r, unsigned off, unsigned soff = 0)
{
    if constexpr (sizeof(S) == 8)
    {
        typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, soff, AUX);
    }
    else if constexpr (sizeof(S) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, soff, AUX);
    else
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, off, soff, AUX);
}

// FP16 storage conversions: the stored value (exact in FP32) times w_i, and
// f*_i / w_i times the scale 2^e rounded to FP16 (nearest even).  The compiler
// may fuse the first product into the sums that follow it, and may do so
// differently in different kernels: the one- and two-nodes-per-lane FP16 paths
// agree to FP16 rounding, not bit for bit.
__device__ __forceinline__ float fp16_in(_Float16 v, float w) { return float(v) * w; }

__device__ __forceinline__ _Float16 fp16_out(float b, float s) { return _Float16(b * s); }

// Layout of the population copies (row-interleaved): in a box, row r = z ny + y
// keeps its planes (the 19 populations, or the 10 moment pieces) as consecutive
// segments of nx values, so element (plane k, x) of row r is at r rb + k kp + x
// with kp = nx and rb = planes nx.  A pull then reads, for each of the few
// upstream rows, one contiguous block of memory instead of 19 planes far apart,
// which keeps HBM streaming close to the rate of a plain copy.
__host__ __device__ __forceinline__ long long pop_index(long long rb, long long kp, int k, long long row, int x)
{
    return row * rb + (long long)k * kp + x;
}

// Addressing of the population copies by the lattice kernels:
//   A_ROW:   all lanes of a wave on one row (tiles whose x extent covers a
//            whole wave): one descriptor per row block in scalar registers,
//            lane offset x, plane offset k kp as the scalar offset operand;
//   A_BOX32: one descriptor at the box start, lane offset r rb + x, scalar
//            offset k kp (boxes under 4 GiB);
//   A_G64:   global accesses with 64-bit per-lane addresses (any box size).
// The descriptors' record counts bound every access to its row block or box.
enum Addr { A_ROW = 0, A_BOX32 = 1, A_G64 = 2 };

// A_ROW: start of row block `row` (32-bit row-block size: 19 planes of a row are far below 4 GiB)
template <class S>
__device__ __forceinline__ const char* row_block(const S* base, long long rb, unsigned row)
{
    return reinterpret_cast<const char*>(base) + (unsigned long long)row * (unsigned(rb) * unsigned(sizeof(S)));
}

template <class S, bool NTL, int ADDR>
__device__ __forceinline__ S load_pop(const S* __restrict__ sb, long long rb, long long kp, unsigned box_bytes, int k,
                                      unsigned row, int x)
{
    constexpr int AUX = NTL ? 2 : 0;
    constexpr unsigned E = sizeof(S);
    if constexpr (ADDR == A_ROW) {
        const unsigned srow = __builtin_amdgcn_readfirstlane(row);
        return bload<S, AUX>(plane_rsrc(row_block(sb, rb, srow), unsigned(rb) * E), unsigned(x) * E,
                             unsigned(k) * unsigned(kp) * E);
    } else if constexpr (ADDR == A_BOX32) {
        return bload<S, AUX>(plane_rsrc(sb, box_bytes), unsigned(pop_index(rb, kp, 0, row, x)) * E,
                             unsigned(k) * unsigned(kp) * E);
    } else {
        const S* p = sb + pop_index(rb, kp, k, row, x);
        if constexpr (NTL)
            return __builtin_nontemporal_load(p);
        else
            return *p;
    }
}

// Non-temporal store of one value (same addressing modes as load_pop).
template <class S, int ADDR>
__device__ __forceinline__ void store_pop(S v, S* __restrict__ db, long long rb, long long kp, unsigned box_bytes, int k,
                                          unsigned row, int x)
{
    constexpr unsigned E = sizeof(S);
    if constexpr (ADDR == A_ROW) {
        const unsigned srow = __builtin_amdgcn_readfirstlane(row);
        bstore<S, 2>(v, plane_rsrc(row_block(db, rb, srow), unsigned(rb) * E), unsigned(x) * E,
                     unsigned(k) * unsigned(kp) * E);
    } else if constexpr (ADDR == A_BOX32) {
        bstore<S, 2>(v, plane_rsrc(db, box_bytes), unsigned(pop_index(rb, kp, 0, row, x)) * E,
                     unsigned(k) * unsigned(kp) * E);
    } else {
        __builtin_nontemporal_store(v, db + pop_index(rb, kp, k, row, x));
    }
}

// FP16 storage, two nodes per lane: the stored values of population k at nodes
// x and x + 1 (x even, nx even) form one 32-bit word, node x in the low half.
// Same addressing modes as load_pop with 32-bit accesses, except that A_ROW takes
// one descriptor per z plane of rows (a pull's upstream rows lie in three planes)
// and puts the row within the plane into the scalar offset: three descriptors
// instead of nine keep the kernel within the scalar registers (a z plane of a box
// is under 4 GiB, checked at set-up).
template <bool NTL, int ADDR>
__device__ __forceinline__ uint32_t load_pair(const _Float16* __restrict__ sb, long long rb, long long kp,
                                              unsigned box_bytes, int ny, int k, unsigned sz, unsigned sy, int x)
{
    constexpr int AUX = NTL ? 2 : 0;
    if constexpr (ADDR == A_ROW) {
        const unsigned z = __builtin_amdgcn_readfirstlane(sz), y = __builtin_amdgcn_readfirstlane(sy);
        const unsigned rbb = unsigned(rb) * 2u;
        return __builtin_amdgcn_raw_buffer_load_b32(plane_rsrc(row_block(sb, rb, z * unsigned(ny)), unsigned(ny) * rbb),
                                                    unsigned(x) * 2u, y * rbb + unsigned(k) * unsigned(kp) * 2u, AUX);
    } else if constexpr (ADDR == A_BOX32) {
        const unsigned row = sz * unsigned(ny) + sy;
        return __builtin_amdgcn_raw_buffer_load_b32(plane_rsrc(sb, box_bytes), unsigned(pop_index(rb, kp, 0, row, x)) * 2u,
                                                    unsigned(k) * unsigned(kp) * 2u, AUX);
    } else {
        const unsigned row = sz * unsigned(ny) + sy;
        const uint32_t* p = reinterpret_cast<const uint32_t*>(sb + pop_index(rb, kp, k, row, x));
        if constexpr (NTL)
            return __builtin_nontemporal_load(p);
        else
            return *p;
    }
}

template <int ADDR>
__device__ __forceinline__ void store_pair(uint32_t v, _Float16* __restrict__ db, long long rb, long long kp,
                                           unsigned box_bytes, int ny, int k, unsigned z, unsigned y, int x)
{
    if constexpr (ADDR == A_ROW) {
        const unsigned sz = __builtin_amdgcn_readfirstlane(z), sy = __builtin_amdgcn_readfirstlane(y);
        const unsigned rbb = unsigned(rb) * 2u;
        __builtin_amdgcn_raw_buffer_store_b32(v, plane_rsrc(row_block(db, rb, sz * unsigned(ny)), unsigned(ny) * rbb),
                                              unsigned(x) * 2u, sy * rbb + unsigned(k) * unsigned(kp) * 2u, 2);
    } else if constexpr (ADDR == A_BOX32) {
        const unsigned row = z * unsigned(ny) + y;
        __builtin_amdgcn_raw_buffer_store_b32(v, plane_rsrc(db, box_bytes), unsigned(pop_index(rb, kp, 0, row, x)) * 2u,
                                              unsigned(k) * unsigned(kp) * 2u, 2);
    } else {
        const unsigned row = z * unsigned(ny) + y;
        __builtin_nontemporal_store(v, reinterpret_cast<uint32_t*>(db + pop_index(rb, kp, k, row, x)));
    }
}

// Pull for two nodes per lane (FP16): word i holds population i of nodes x and
// x + 1, gathered from x - c_i and x + 1 - c_i.  A population moving in +x needs
// the upper half of the pair to the left, one moving in -x the lower half of the
// pair to the right.  With a whole wave on one tile row (LX >= 64) the neighbour
// pairs come from the adjacent lanes by a DPP wave shift; the wave's first lane
// takes the pair left of the wave, and its last lane (or the lane at the end of
// the box row, in a ragged tile) the pair right of it, each from one load at a
// wave-uniform address.  All loads are issued before the shifts, which wait for
// them.  Narrower tiles load each lane's neighbour pair directly.  x is the
// lane's even node, xl / xr the even nodes of the pairs to its left and right
// (periodic wrap).
template <int LX, bool NTL, int ADDR>
__device__ __forceinline__ void pull_pairs(const _Float16* __restrict__ sb, long long rb, long long kp, unsigned box_bytes,
                                           int ny, int nx, int x, int xl, int xr, int y, int z, int ym, int yp, int zm,
                                           int zp, uint32_t (&w)[NQ])
{
    uint32_t own[NQ], edge[NQ];
    const int lane = threadIdx.x & 63;
    // wave-uniform edge pairs (used when LX >= 64): left of lane 0, right of lane 63
    const int el = __builtin_amdgcn_readfirstlane(xl);
    const int er = __builtin_amdgcn_readlane(xr, 63);
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const int cx = cvel(i, 0), cy = cvel(i, 1), cz = cvel(i, 2);
        const int sy = cy > 0 ? ym : (cy < 0 ? yp : y);
        const int sz = cz > 0 ? zm : (cz < 0 ? zp : z);
        own[i] = load_pair<NTL, ADDR>(sb, rb, kp, box_bytes, ny, i, unsigned(sz), unsigned(sy), x);
        if (cx != 0) {
            const int xe = LX >= 64 ? (cx > 0 ? el : er) : (cx > 0 ? xl : xr);
            edge[i] = load_pair<NTL, ADDR>(sb, rb, kp, box_bytes, ny, i, unsigned(sz), unsigned(sy), xe);
        }
    }
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const int cx = cvel(i, 0);
        if (cx == 0) {
            w[i] = own[i];
        } else if (cx > 0) {
            uint32_t prev = edge[i];
            if constexpr (LX >= 64) {
                // wave_shr:1; lane 0 has no source lane and, with bound_ctrl off, keeps the edge word
                prev = uint32_t(__builtin_amdgcn_update_dpp(int(edge[i]), int(own[i]), 0x138, 0xf, 0xf, false));
            }
            w[i] = __builtin_amdgcn_alignbit(own[i], prev, 16);    // (prev.hi, own.lo)
        } else {
            uint32_t next = edge[i];
            if constexpr (LX >= 64) {
                // wave_shl:1; lane 63 likewise.  In a tile row that runs past nx the lanes past the
                // end hold x = 0, so the last node pair's right neighbour is the periodic wrap.
                next = uint32_t(__builtin_amdgcn_update_dpp(int(edge[i]), int(own[i]), 0x130, 0xf, 0xf, false));
            }
            w[i] = __builtin_amdgcn_alignbit(next, own[i], 16);    // (own.hi, next.lo)
        }
    }
}

// The 19 pre-collision populations of node (x, y, z) as deviations (for FP16
// storage the stored (deviation / w_i) 2^e times w_i sc, sc = 2^-e for the
// deviation itself), pulled from the post-collision data of the upstream nodes
// x - c_i.  xm/xp etc. are the periodic neighbours of x, y, z.  The populations layout reads one value per
// direction; the moment layout rebuilds each population from the upstream
// node's stored bracket pieces.
template <int ST, bool NTL, int ADDR>
__device__ __forceinline__ void pull_node(const typename StoreT<ST>::S* __restrict__ sb, long long rb, long long kp,
                                          unsigned box_bytes, int ny, int x, int y, int z, int xm, int xp, int ym,
                                          int yp, int zm, int zp, typename StoreT<ST>::T (&f)[NQ], float sc = 1.0f)
{
    using S = typename StoreT<ST>::S;
    using T = typename StoreT<ST>::T;
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
        const int cx = cvel(i, 0), cy = cvel(i, 1), cz = cvel(i, 2);
        const int sx = cx > 0 ? xm : (cx < 0 ? xp : x);
        const int sy = cy > 0 ? ym : (cy < 0 ? yp : y);
        const int sz = cz > 0 ? zm : (cz < 0 ? zp : z);
        const unsigned row = unsigned(sz) * unsigned(ny) + unsigned(sy);
        auto piece = [&](int k) -> T {
            return T(load_pop<S, NTL, ADDR>(sb, rb, kp, box_bytes, k, row, sx));
        };
        if constexpr (ST == ST_MOM32) {
            T br = piece(MP_R0);
            if (cx != 0) br += (cx > 0 ? piece(MP_AX) : -piece(MP_AX)) + piece(MP_BXX);
            if (cy != 0) br += (cy > 0 ? piece(MP_AY) : -piece(MP_AY)) + piece(MP_BYY);
            if (cz != 0) br += (cz > 0 ? piece(MP_AZ) : -piece(MP_AZ)) + piece(MP_BZZ);
            if (cx * cy != 0) br += cx * cy > 0 ? piece(MP_BXY) : -piece(MP_BXY);
            if (cx * cz != 0) br += cx * cz > 0 ? piece(MP_BXZ) : -piece(MP_BXZ);
            if (cy * cz != 0) br += cy * cz > 0 ? piece(MP_BYZ) : -piece(MP_BYZ);
            f[i] = T(wgt(i)) * br;
        } else if constexpr (ST == ST_FP16) {
            f[i] = fp16_in(load_pop<S, NTL, ADDR>(sb, rb, kp, box_bytes, i, row, sx), float(wgt(i)) * sc);
        } else {
            f[i] = piece(i);
        }
    }
}

// Wrap r into [0, L).
__device__ __forceinline__ double wrap_pos(double r, double L)
{
    if (r >= 0.0 && r < L) return r + 0.0;   // the usual case (+ 0.0: a negative zero becomes +0)
    r -= L * floor(r / L);
    if (r >= L) r -= L;
    if (r < 0.0) r = 0.0;
    return r;
}

}  // namespace lbm

// Lattice kernels: the fused forced-MRT step and the moment / diagnostic
// passes that share its per-node arithmetic.  Templates and launchers only;
// each storage mode is instantiated by its own lbm_lattice_<storage>.hip.
//
// One thread per node, one 256-thread block per tile of TX x TY x TZ nodes
// (x fastest, one wave64 per x-row segment).  The step is a pull scheme:
// node x gathers population i from x - c_i of the source copy (the
// propagation of Sec. II), collides in registers and writes its own 19
// post-collision populations to the destination copy.  Populations are kept
// as deviations from w_i rho0; the FP16 mode stores (deviation / w_i) * 2^e.
//
// Collision, per node (Eq. fiexp and the A, B that follow it; ghosts projected
// out, every stress mode relaxed with omega = 1/(tau + 1/2)):
//   drho = sum df_i,  j = sum df_i c_i,  S = sum df_i (c_i c_i - I/3)
//   rho = rho0 + drho,  u = (j + g/2) / rho              (Eq. macrovariables2)
//   A = j + g
//   B = S - omega (S - rho u u - tau (u g + g u))       (sign from Eq. mrtlbe)
//   df*_i = w_i [ drho + 3 A.c_i + 9/2 B:(c_i c_i - I/3) ]
// g is the force density spread from the tile's points with the Peskin kernel
// (Sec. III) plus the optional uniform counter-force; u feeds the per-(tile,
// point) interpolation partial sums of Sec. IV.  The general operators (BGK,
// MRT with bulk and ghost rates) and the thermal step add to this the ghost
// part of the pulled state and the mode noise (COLL below).
#pragma once

#include <hip/hip_ext.h>

#include "lbm_device.h"
#include "lbm_internal.h"
#include "lbm_noise.h"

namespace lbm {

enum Mode { M_STEP = 0, M_MOMENTS = 1, M_DIAG = 2 };


// VAR bit 0: global loads/stores with 64-bit per-lane addresses instead of
// raw buffer accesses (scalar descriptor + 32-bit lane offset).
// VAR bit 1: cached instead of non-temporal population loads.
// COLL: 1 = general collision of Eq. mrtlbe (bulk mode at its own rate, ghost
// moments multiplied by kappa_g instead of projected out); 2 = the same plus
// thermal noise on the fifteen non-conserved modes, drawn for step *tin.
template <int ST, int TX, int TY, int TZ, int MODE, int VAR, int COLL = 0, int NPL = 1>
__device__ __forceinline__ void lattice_tile(const Geom& G, const int tile,
                                             const typename StoreT<ST>::S* __restrict__ src,
                                             typename StoreT<ST>::S* __restrict__ dst,
                                             const BoxDev* __restrict__ boxes,
                                             const int* __restrict__ toff, const int* __restrict__ tlist,
                                             const PRec<typename StoreT<ST>::T>* __restrict__ rec,
                                             double* __restrict__ out0, double* __restrict__ out1,
                                             const unsigned long long* __restrict__ tin)
{
    using S = typename StoreT<ST>::S;
    using T = typename StoreT<ST>::T;
    static_assert(TX * TY * TZ == BLOCK, "tiles of BLOCK nodes");
    // NPL = 2: each lane takes the two adjacent nodes x, x + 1 (FP16 storage, nx even),
    // half as many threads per tile
    static_assert(NPL == 1 || (NPL == 2 && ST == ST_FP16 && MODE == M_STEP), "two nodes per lane: FP16 step only");
    constexpr int LX = TX / NPL;              // lanes along x in a tile row
    constexpr int NW = BLOCK / NPL / 64;      // waves per block

    // (the divisions by the tile counts use multipliers set on the host: a 64-bit product and a
    // shift in the scalar unit, with no reciprocal to set up in the kernel)
    const unsigned t0 = unsigned(tile);
    const unsigned t1 = div_magic(t0, G.mtx, G.stx), t2 = div_magic(t1, G.mty, G.sty);
    const unsigned t3 = div_magic(t2, G.mtz, G.stz);
    const int itx = int(t0 - t1 * unsigned(G.ntx));
    const int ity = int(t1 - t2 * unsigned(G.nty));
    const int itz = int(t2 - t3 * unsigned(G.ntz));
    const int box = int(t3);
    // a tile row of at least 64 lanes puts each wave on one row: y and z are then wave-uniform
    // and live in scalar registers (so do the upstream row indices of the pull)
    const int tid_w = LX >= 64 ? __builtin_amdgcn_readfirstlane(int(threadIdx.x)) : int(threadIdx.x);
    const int lx = threadIdx.x % LX, ly = (tid_w / LX) % TY, lz = tid_w / (LX * TY);
    const int x0 = itx * TX + lx * NPL, y0 = ity * TY + ly, z0 = itz * TZ + lz;
    const bool valid = (x0 < G.nx) & (y0 < G.ny) & (z0 < G.nz);
    // threads past a ragged edge work on an in-range node and contribute nothing: the clamped
    // one, or with two nodes per lane (nx even) x = 0, the periodic wrap that the lane before
    // them takes as its right neighbour
    const int x = NPL == 2 ? (x0 < G.nx ? x0 : 0) : min(x0, G.nx - NPL), y = min(y0, G.ny - 1), z = min(z0, G.nz - 1);
    const int xm = x == 0 ? G.nx - 1 : x - 1, xp = x + 1 == G.nx ? 0 : x + 1;
    const int ym = y == 0 ? G.ny - 1 : y - 1, yp = y + 1 == G.ny ? 0 : y + 1;
    const int zm = z == 0 ? G.nz - 1 : z - 1, zp = z + 1 == G.nz ? 0 : z + 1;

    const BoxDev& B = boxes[box];
    const S* sb = src + (long long)box * G.sbox;

    // ---- pull: population i at x comes from x - c_i
    // Addressing (see load_pop): a tile row of at least 64 lanes keeps each wave on one row;
    // narrower tiles address from the box start (boxes under 4 GiB, checked at set-up);
    // variant bit 0 uses 64-bit global addresses.
    constexpr bool WIDE = (VAR & 1);
    constexpr int ADDR = WIDE ? A_G64 : (LX >= 64 ? A_ROW : A_BOX32);
    // moment pieces are re-read by up to 18 neighbours: always cached loads
    constexpr bool NTL = !(VAR & 2) && ST != ST_MOM32;
    const unsigned box_bytes = unsigned(G.sbox * (long long)sizeof(S));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    [[maybe_unused]] uint32_t wpair[NPL == 2 ? NQ : 1];
    // FP16: stored values are (deviation / w_i) 2^e; the conversion multiplies by w_i 2^-e (exact:
    // a power of two times w_i), so the moments come out in deviation units
    [[maybe_unused]] const float sc = ST == ST_FP16 ? (MODE == M_STEP ? B.s_in : ldexpf(1.0f, -B.e_data)) : 1.0f;
    T f[NQ];
    if constexpr (NPL == 2) {
        const int xl = x == 0 ? G.nx - 2 : x - 2, xr = x + 2 == G.nx ? 0 : x + 2;
        pull_pairs<LX, NTL, ADDR>(reinterpret_cast<const _Float16*>(sb), G.rb, G.kp, box_bytes, G.ny, G.nx, x, xl, xr,
                                  y, z, ym, yp, zm, zp, wpair);
    } else {
        pull_node<ST, NTL, ADDR>(sb, G.rb, G.kp, box_bytes, G.ny, x, y, z, xm, xp, ym, yp, zm, zp, f, sc);
    }

    int k0 = 0, k1 = 0;         // the tile's entries in the point lists (read below)
    S* db = dst + (long long)box * G.sbox;
    const unsigned row = unsigned(z) * unsigned(G.ny) + unsigned(y);
    typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
    [[maybe_unused]] half2_t opair[NPL == 2 ? NQ : 1];
    bool bad = false;
    T mx = 0;                     // FP16: largest |f*_i / w_i| of the lane's nodes
    T uxs[NPL], uys[NPL], uzs[NPL];
    [[maybe_unused]] T pc[NPL][MP_N];   // two FP16 nodes, projected collision: each node's ten pieces
    const T gcx = T(B.gc[0]), gcy = T(B.gc[1]), gcz = T(B.gc[2]);   // the box's counter-force density
    const T rho0 = T(G.rho0), tau = T(B.tau), om = T(B.omega);         // converted once per lane

    // ---- per node of the lane: moments, force, collision, post-collision values
#pragma unroll
    for (int h = 0; h < NPL; ++h) {
        const int xh = x + h;
        // projected collision on two FP16 nodes per lane: moments straight from the stored halves
        constexpr bool RAW = NPL == 2 && COLL == 0;
        if constexpr (NPL == 2 && !RAW) {
            // FP16 value of node xh (low half: x, high half: x + 1), converted exactly, then weighted
#pragma unroll
            for (int i = 0; i < NQ; ++i) {
                const uint32_t bits = h == 0 ? (wpair[i] & 0xffffu) : (wpair[i] >> 16);
                f[i] = fp16_in(__builtin_bit_cast(_Float16, uint16_t(bits)), float(wgt(i)) * sc);
            }
        }

        // ---- moments (10 values), over opposite pairs (i, i+1): the pair sum feeds the even
        // moments (mass, second moments), the difference the odd ones (momentum).  Each sum
        // starts at its first term (no addition of zero).
        T drho, jx = 0, jy = 0, jz = 0, pxx = 0, pyy = 0, pzz = 0, pxy = 0, pxz = 0, pyz = 0;
        if constexpr (RAW) {
            // Opposite populations share their weight w_i = k_i / 36 (k = 12 rest, 2 axis, 1
            // diagonal), so each moment is (2^-e / 36) times a sum over pairs of the stored values'
            // pair sums and differences, the axis pair counted twice.  A pair sum or difference of
            // two FP16 halves is one mixed-precision multiply-add (by the unit G.one).
            const T one = T(G.one);
            auto hv = [&](int i) {
                const half2_t v = __builtin_bit_cast(half2_t, wpair[i]);
                return h == 0 ? v.x : v.y;
            };
            // per moment: the axis term (at most one per moment but three for the mass) and the
            // diagonal terms, each accumulated from its first term
            T ra = 0, rd = 0, xa = 0, xd = 0, ya = 0, yd = 0, za = 0, zd = 0;
            T qxa = 0, qxd = 0, qya = 0, qyd = 0, qza = 0, qzd = 0;
            bool s_ra = false, s_rd = false, s_xa = false, s_xd = false, s_ya = false, s_yd = false, s_za = false,
                 s_zd = false, s_qxa = false, s_qxd = false, s_qya = false, s_qyd = false, s_qza = false,
                 s_qzd = false, s_pxy = false, s_pxz = false, s_pyz = false;
#pragma unroll
            for (int i = 1; i < NQ; i += 2) {
                const T sm = __builtin_fmaf(float(hv(i)), one, float(hv(i + 1)));
                const T df = __builtin_fmaf(float(hv(i)), one, -float(hv(i + 1)));
                const int cx = cvel(i, 0), cy = cvel(i, 1), cz = cvel(i, 2);
                const bool axis = cx * cx + cy * cy + cz * cz == 1;
                if (axis) acc_first(ra, s_ra, sm); else acc_first(rd, s_rd, sm);
                if (cx != 0) {
                    if (axis) { acc_first(xa, s_xa, cx > 0 ? df : -df); acc_first(qxa, s_qxa, sm); }
                    else { acc_first(xd, s_xd, cx > 0 ? df : -df); acc_first(qxd, s_qxd, sm); }
                }
                if (cy != 0) {
                    if (axis) { acc_first(ya, s_ya, cy > 0 ? df : -df); acc_first(qya, s_qya, sm); }
                    else { acc_first(yd, s_yd, cy > 0 ? df : -df); acc_first(qyd, s_qyd, sm); }
                }
                if (cz != 0) {
                    if (axis) { acc_first(za, s_za, cz > 0 ? df : -df); acc_first(qza, s_qza, sm); }
                    else { acc_first(zd, s_zd, cz > 0 ? df : -df); acc_first(qzd, s_qzd, sm); }
                }
                if (cx * cy != 0) acc_first(pxy, s_pxy, cx * cy > 0 ? sm : -sm);
                if (cx * cz != 0) acc_first(pxz, s_pxz, cx * cz > 0 ? sm : -sm);
                if (cy * cz != 0) acc_first(pyz, s_pyz, cy * cz > 0 ? sm : -sm);
            }
            const T u = sc * T(1.0 / 36.0);   // 2^-e / 36: exact enough (one rounding of a constant)
            drho = u * __builtin_fmaf(float(hv(0)), T(12), __builtin_fmaf(T(2), ra, rd));
            jx = u * __builtin_fmaf(T(2), xa, xd);
            jy = u * __builtin_fmaf(T(2), ya, yd);
            jz = u * __builtin_fmaf(T(2), za, zd);
            pxx = u * __builtin_fmaf(T(2), qxa, qxd);
            pyy = u * __builtin_fmaf(T(2), qya, qyd);
            pzz = u * __builtin_fmaf(T(2), qza, qzd);
            pxy *= u;
            pxz *= u;
            pyz *= u;
        } else {
            drho = f[0];
            bool s_jx = false, s_jy = false, s_jz = false, s_pxx = false, s_pyy = false, s_pzz = false,
                 s_pxy = false, s_pxz = false, s_pyz = false;
#pragma unroll
            for (int i = 1; i < NQ; i += 2) {
                const T sm = f[i] + f[i + 1], df = f[i] - f[i + 1];
                const int cx = cvel(i, 0), cy = cvel(i, 1), cz = cvel(i, 2);
                drho += sm;
                if (cx != 0) { acc_first(jx, s_jx, cx > 0 ? df : -df); acc_first(pxx, s_pxx, sm); }
                if (cy != 0) { acc_first(jy, s_jy, cy > 0 ? df : -df); acc_first(pyy, s_pyy, sm); }
                if (cz != 0) { acc_first(jz, s_jz, cz > 0 ? df : -df); acc_first(pzz, s_pzz, sm); }
                if (cx * cy != 0) acc_first(pxy, s_pxy, cx * cy > 0 ? sm : -sm);
                if (cx * cz != 0) acc_first(pxz, s_pxz, cx * cz > 0 ? sm : -sm);
                if (cy * cz != 0) acc_first(pyz, s_pyz, cy * cz > 0 ? sm : -sm);
            }
        }

        // ---- force density at this node: counter-force + the tile's points
        T gx = gcx, gy = gcy, gz = gcz;
        if (h == 0 && toff) {
            k0 = toff[tile];
            k1 = toff[tile + 1];
        }
        for (int k = k0; k < k1; ++k) {
            const PRec<T>& r = rec[pk_point(tlist[k])];
            // rows the point's stencil misses take nothing from it: skip them (a scalar branch
            // when y and z are wave-uniform; otherwise waves whose lanes all miss skip it)
            int dy = y - r.by, dz = z - r.bz;
            if (dy < 0) dy += G.ny;
            if (dz < 0) dz += G.nz;
            if (dy > 3 || dz > 3) continue;
            const T w = stencil_w<T>(xh, r.bx, G.nx, r.wx) * stencil_w<T>(y, r.by, G.ny, r.wy) *
                        stencil_w<T>(z, r.bz, G.nz, r.wz);
            gx += r.f[0] * w;
            gy += r.f[1] * w;
            gz += r.f[2] * w;
        }

        const T rho = rho0 + drho;
        // FP16 storage: the hardware reciprocal (1 ulp), far below the storage's rounding
        T ir;
        if constexpr (ST == ST_FP16)
            ir = __builtin_amdgcn_rcpf(rho);
        else
            ir = T(1) / rho;
        // rho u = j + g/2 (Eq. macrovariables2)
        const T hx = jx + T(0.5) * gx, hy = jy + T(0.5) * gy, hz = jz + T(0.5) * gz;
        const T ux = hx * ir, uy = hy * ir, uz = hz * ir;

        if constexpr (MODE == M_MOMENTS) {
            if (valid) {
                const long long n = ((long long)z * G.ny + y) * G.nx + x;
                if (out0) out0[(long long)box * G.N + n] = G.rho0 + double(drho);
                out1[((long long)box * 3 + 0) * G.N + n] = double(ux);
                out1[((long long)box * 3 + 1) * G.N + n] = double(uy);
                out1[((long long)box * 3 + 2) * G.N + n] = double(uz);
            }
            return;
        }

        if constexpr (MODE == M_DIAG) {
            const T chk = drho + jx + jy + jz + pxx + pyy + pzz + pxy + pxz + pyz + gx + gy + gz;
            const bool nonfin = !(fabs(chk) <= T(sizeof(T) == 4 ? 3.0e38 : 1.0e300));
            double v[LBD_N];
            const double X = x, Y = y, Z = z;
            v[0] = drho; v[1] = jx; v[2] = jy; v[3] = jz;
            v[4] = gx; v[5] = gy; v[6] = gz;
            v[7] = Y * double(gz) - Z * double(gy);
            v[8] = Z * double(gx) - X * double(gz);
            v[9] = X * double(gy) - Y * double(gx);
            v[10] = sqrt(double(ux) * ux + double(uy) * uy + double(uz) * uz);
            v[11] = nonfin ? 1.0 : 0.0;
            v[12] = rho > T(0) ? 0.0 : 1.0;   // non-positive density (NaN counts under 11, not here)
            if (nonfin) v[12] = 0.0;
            __shared__ double red[4][LBD_N];
#pragma unroll
            for (int c = 0; c < LBD_N; ++c) {
                double a = valid ? v[c] : 0.0;
                if (c == 10) {
                    if (!(a == a)) a = 0.0;  // max ignores NaN; the count reports it
                    a = wave_max(a);
                } else {
                    a = wave_sum(a);
                }
                if (lane == 0) red[wave][c] = a;
            }
            __syncthreads();
            if (threadIdx.x < LBD_N) {
                const int c = threadIdx.x;
                double a;
                if (c == 10)
                    a = fmax(fmax(red[0][c], red[1][c]), fmax(red[2][c], red[3][c]));
                else
                    a = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
                out0[(long long)tile * LBD_N + c] = a;
            }
            return;
        }

        // ---- M_STEP: collide
        const T ax = jx + gx, ay = jy + gy, az = jz + gz;
        const T third = T(1.0 / 3.0);
        const T sxx = pxx - drho * third, syy = pyy - drho * third, szz = pzz - drho * third;
        T br[NQ];   // post-collision f*_i / w_i
        if constexpr (COLL && ST != ST_MOM32) {
            // ghost part of the pulled state (deviation minus its projection onto 1, c, Q),
            // carried over with factor kappa_g, in units of w_i; taken first so that the pulled
            // populations are dead before the collision
            const T kg = T(B.kappa_g);
            const T hbase = drho - T(1.5) * (sxx + syy + szz);
#pragma unroll
            for (int i = 0; i < NQ; ++i) {
                const int cx = cvel(i, 0), cy = cvel(i, 1), cz = cvel(i, 2);
                T a = 0, q = 0;
                if (cx != 0) { a += cx > 0 ? jx : -jx; q += sxx; }
                if (cy != 0) { a += cy > 0 ? jy : -jy; q += syy; }
                if (cz != 0) { a += cz > 0 ? jz : -jz; q += szz; }
                if (cx * cy != 0) q += cx * cy > 0 ? T(2) * pxy : T(-2) * pxy;
                if (cx * cz != 0) q += cx * cz > 0 ? T(2) * pxz : T(-2) * pxz;
                if (cy * cz != 0) q += cy * cz > 0 ? T(2) * pyz : T(-2) * pyz;
                const T hb = hbase + T(3) * a + T(4.5) * q;
                const T inv_w = i == 0 ? T(3) : (cx * cx + cy * cy + cz * cz == 1 ? T(18) : T(36));
                br[i] = kg * (f[i] * inv_w - hb);
            }
        }
        // the equilibrium and forcing part of the stress, rho u_a u_b + tau (u_a g_b + g_a u_b), as
        // u_b (rho u_a + tau g_a) + u_a tau g_b with rho u_a = h_a
        const T tgx = tau * gx, tgy = tau * gy, tgz = tau * gz;
        const T qx = hx + tgx, qy = hy + tgy, qz = hz + tgz;
        T Bxx, Byy, Bzz;
        if constexpr (COLL) {
            // shear drivers of the diagonal; their trace relaxes at omega_b instead (bulk mode)
            const T dxx = sxx - ux * (qx + tgx);
            const T dyy = syy - uy * (qy + tgy);
            const T dzz = szz - uz * (qz + tgz);
            const T trs = (dxx + dyy + dzz) * third;
            const T tb = T(B.tau_b), omb = T(B.omega_b);
            const T trb = (sxx + syy + szz - rho * (ux * ux + uy * uy + uz * uz) -
                           tb * (T(2) * (ux * gx + uy * gy + uz * gz))) * third;
            Bxx = sxx - om * (dxx - trs) - omb * trb;
            Byy = syy - om * (dyy - trs) - omb * trb;
            Bzz = szz - om * (dzz - trs) - omb * trb;
        } else {
            Bxx = sxx - om * (sxx - ux * (qx + tgx));
            Byy = syy - om * (syy - uy * (qy + tgy));
            Bzz = szz - om * (szz - uz * (qz + tgz));
        }
        const T Bxy = pxy - om * (pxy - (uy * qx + ux * tgy));
        const T Bxz = pxz - om * (pxz - (uz * qx + ux * tgz));
        const T Byz = pyz - om * (pyz - (uz * qy + uy * tgz));
        // FP16, two nodes per lane, projected operator: the pieces below carry the output scale 2^e
        // (exact), so the rebuilt brackets are the values to round and each pair of nodes is
        // converted by one packing conversion without a multiply (one node per lane converts
        // with a mixed-precision multiply, where the scale costs nothing)
        constexpr bool FOLD = ST == ST_FP16 && COLL == 0 && NPL == 2;
        const T so = FOLD ? T(B.s_out) : T(1);
        T base = FOLD ? so * drho - (T(1.5) * so) * (Bxx + Byy + Bzz) : drho - T(1.5) * (Bxx + Byy + Bzz);

        // f*_i / w_i = base + c_i.(3A) + sum_a c_ia^2 (9/2) B_aa + sum_{a<b} c_ia c_ib 9 B_ab: for an
        // opposite pair the even part is shared and the odd part (3A.c_i) changes sign
        const T a3x = (T(3) * so) * ax, a3y = (T(3) * so) * ay, a3z = (T(3) * so) * az;
        T bxx = (T(4.5) * so) * Bxx, byy = (T(4.5) * so) * Byy, bzz = (T(4.5) * so) * Bzz;
        T bxy = (T(9) * so) * Bxy, bxz = (T(9) * so) * Bxz, byz = (T(9) * so) * Byz;
        [[maybe_unused]] const float s_store = FOLD ? 1.0f : B.s_out;   // scale still to apply at the store

        // thermal increment w_i sum_k e_k(c_i) phi_k / b_k, <phi_k^2> = mu rho b_k (1 - gamma_k^2), in
        // units of w_i: amp[k] = phi_k / b_k.  Philox call j gives the normals of modes 4j .. 4j+3.
        // The bulk and shear modes fold into the pieces above (stress_modes_fold); the ghosts are
        // added per opposite pair after the rebuild, as an even and an odd part.
        [[maybe_unused]] T amp[16];
        [[maybe_unused]] uint32_t node = 0;
        [[maybe_unused]] unsigned long long tstep = 0;
        auto draw = [&](int j) {
            const Philox4 q = node_draw(node, uint32_t(box), tstep, uint32_t(j), G.seed_lo, G.seed_hi);
            T r[4];
            box_muller<T>(q.v[0], q.v[1], r[0], r[1]);
            box_muller<T>(q.v[2], q.v[3], r[2], r[3]);
            const T sr = noise_sqrt(rho);
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int k = 4 * j + m;
                if (k >= 15) continue;
                const T nzk = T(k == 0 ? B.nz_b : (k < 6 ? B.nz_s : B.nz_g));
                amp[k] = sr * nzk * T(1.0 / __builtin_sqrt(mode_norm(k))) * r[m];
            }
        };
        if constexpr (COLL == 2 && ST != ST_MOM32) {
            tstep = *tin;
            node = (unsigned(z) * unsigned(G.ny) + unsigned(y)) * unsigned(G.nx) + unsigned(xh);
            draw(0);
            draw(1);
            base -= amp[0];
            bxx += amp[0] + T(2) * amp[1];
            byy += amp[0] - amp[1] + amp[2];
            bzz += amp[0] - amp[1] - amp[2];
            bxy += amp[3];
            bxz += amp[4];
            byz += amp[5];
        }
        const T piece[MP_N] = {base, a3x, a3y, a3z, bxx, byy, bzz, bxy, bxz, byz};
        if constexpr (RAW) {
            // both nodes' outputs are rebuilt from their pieces after the loop, one packed word at a time
#pragma unroll
            for (int k = 0; k < MP_N; ++k) pc[h][k] = piece[k];
        }
        constexpr bool GHOST = COLL && ST != ST_MOM32;
        // with the ghost part already in br: br + (ev +- od), the same sum as (ev +- od) + br
        br[0] = GHOST ? br[0] + base : base;
#pragma unroll
        for (int i = 1; i < NQ; i += 2) {
            T bp, bm;
            rebuild_pair(piece, i, bp, bm);
            br[i] = GHOST ? br[i] + bp : bp;
            br[i + 1] = GHOST ? br[i + 1] + bm : bm;
        }
        if constexpr (COLL == 2 && ST != ST_MOM32) {
            draw(2);
            draw(3);
            br[0] += amp[12];     // the only ghost that is non-zero at rest (e_12(0) = 1)
#pragma unroll
            for (int i = 1; i < NQ; i += 2) {
                T ev = 0, od = 0;
#pragma unroll
                for (int k = 6; k < 15; ++k) {
                    const int e = emode(k, i);
                    if (e == 0) continue;
                    if (mode_even(k))
                        ev += T(e) * amp[k];
                    else
                        od += T(e) * amp[k];
                }
                br[i] += ev + od;
                br[i + 1] += ev - od;
            }
        }

        // ---- health of this node: non-finite moments or forces
        {
            // FP16 populations are bounded (|stored| <= 65504), so a non-finite one always reaches drho;
            // the other storages also check the sums that could overflow on their own
            const T chk = ST == ST_FP16 ? drho + gx + gy + gz : drho + jx + jy + jz + pxx + pyy + pzz + gx + gy + gz;
            bad = bad || (valid && !(fabs(chk) <= T(sizeof(T) == 4 ? 3.0e38 : 1.0e300)));
        }

        // ---- store the post-collision state of this node (two nodes per lane: packed below)
        if constexpr (RAW) {
        } else if constexpr (NPL == 2) {
#pragma unroll
            for (int i = 0; i < NQ; ++i) {
                if (h == 0)
                    opair[i].x = fp16_out(br[i], s_store);
                else
                    opair[i].y = fp16_out(br[i], s_store);
            }
        } else if (valid) {
            if constexpr (ST == ST_MOM32) {
                const T piece[MP_N] = {base, a3x, a3y, a3z, bxx, byy, bzz, bxy, bxz, byz};
#pragma unroll
                for (int k = 0; k < MP_N; ++k) store_pop<S, ADDR>(piece[k], db, G.rb, G.kp, box_bytes, k, row, x);
            } else {
#pragma unroll
                for (int i = 0; i < NQ; ++i) {
                    S v;
                    if constexpr (ST == ST_FP16)
                        v = fp16_out(br[i], s_store);
                    else
                        v = S(T(wgt(i)) * br[i]);
                    store_pop<S, ADDR>(v, db, G.rb, G.kp, box_bytes, i, row, x);
                }
            }
        }

        // ---- FP16: the largest bracket magnitude (with FOLD already times 2^e), for the range
        // check and the rescaling
        if constexpr (ST == ST_FP16 && !RAW) {
#pragma unroll
            for (int i = 0; i < NQ; ++i) mx = fmax(mx, fabs(br[i]));
        }
        uxs[h] = ux;
        uys[h] = uy;
        uzs[h] = uz;
    }   // nodes of the lane

    if constexpr (NPL == 2 && COLL == 0) {
        // the two nodes' post-collision values (already times 2^e), word by word: rebuilt from the
        // pieces, packed, folded into the lane's maximum and stored, so that only the pieces stay live
        if (valid) {
            auto put = [&](int i, T v0, T v1) {
                half2_t w;
                w.x = fp16_out(v0, 1.0f);
                w.y = fp16_out(v1, 1.0f);
                mx = fmax(fmax(mx, fabs(v0)), fabs(v1));   // one v_max3
                store_pair<ADDR>(__builtin_bit_cast(uint32_t, w), reinterpret_cast<_Float16*>(db), G.rb, G.kp,
                                 box_bytes, G.ny, i, unsigned(z), unsigned(y), x);
            };
            put(0, pc[0][MP_R0], pc[1][MP_R0]);
#pragma unroll
            for (int i = 1; i < NQ; i += 2) {
                T p0, m0, p1, m1;
                rebuild_pair(pc[0], i, p0, m0);
                rebuild_pair(pc[1], i, p1, m1);
                put(i, p0, p1);
                put(i + 1, m0, m1);
            }
        }
    } else if constexpr (NPL == 2) {
        if (valid) {
#pragma unroll
            for (int i = 0; i < NQ; ++i)
                store_pair<ADDR>(__builtin_bit_cast(uint32_t, opair[i]), reinterpret_cast<_Float16*>(db), G.rb, G.kp,
                                 box_bytes, G.ny, i, unsigned(z), unsigned(y), x);
        }
    }
    if constexpr (ST == ST_FP16) {
        constexpr bool FOLD = COLL == 0 && NPL == 2;
        T m = valid ? mx : T(0);
        bad = bad || ((FOLD ? m : m * B.s_out) > T(65504));
        m = wave_max_nonneg(m);   // m = |f*| magnitudes: non-negative
        // the largest |f*_i / w_i|, without the scale: 1 / 2^e (exact) from the bits of 2^e
        if (FOLD) m *= __uint_as_float(0x7f000000u - __float_as_uint(B.s_out));
        if (G.smax) {
            // one box: each wave into the box's maximum (non-negative floats order as their bit
            // patterns), no exchange between the block's waves
            if (lane == 0) atomicMax(G.smax + (tile % SMAX_SLOTS) * SMAX_STRIDE, __float_as_uint(m));
        } else {
            // per-tile maximum; the per-box reduction happens before the next step
            __shared__ float wm[NW];
            if (lane == 0) wm[wave] = m;
            __syncthreads();
            if (threadIdx.x == 0) {
                float t = wm[0];
#pragma unroll
                for (int q = 1; q < NW; ++q) t = fmaxf(t, wm[q]);
                ((float*)out1)[tile] = t;
            }
            __syncthreads();   // wm is rewritten by the block's next tile
        }
    }
    if (__any(bad) && lane == 0) atomicOr(&G.nf[box], 1);

    // ---- interpolation partial sums: sum over this tile's nodes of u * deltaP(x - R)
    // u of the tile's nodes goes to LDS; wave w then takes the tile's points w, w + NW, ...,
    // lane l standing for stencil node (l & 3, (l >> 2) & 3, l >> 4) of the point, and one
    // wave reduction per component gives the point's partial.
    if (k1 > k0) {
        __shared__ T su[3][BLOCK];
#pragma unroll
        for (int h = 0; h < NPL; ++h) {
            // node index in the tile
            const int li = NPL == 1 ? int(threadIdx.x) : lx * NPL + h + TX * (ly + TY * lz);
            su[0][li] = valid ? uxs[h] : T(0);
            su[1][li] = valid ? uys[h] : T(0);
            su[2][li] = valid ? uzs[h] : T(0);
        }
        __syncthreads();
        const int dx = lane & 3, dy = (lane >> 2) & 3, dz = lane >> 4;
        const int x0 = itx * TX, y0 = ity * TY, z0 = itz * TZ;
        for (int kk = k0 + wave; kk < k1; kk += NW) {
            const int ent = tlist[kk];
            const PRec<T>& r = rec[pk_point(ent)];
            int gx = r.bx + dx, gy = r.by + dy, gz = r.bz + dz;
            if (gx >= G.nx) gx -= G.nx;
            if (gy >= G.ny) gy -= G.ny;
            if (gz >= G.nz) gz -= G.nz;
            const int lx2 = gx - x0, ly2 = gy - y0, lz2 = gz - z0;
            const bool in = unsigned(lx2) < unsigned(TX) && unsigned(ly2) < unsigned(TY) && unsigned(lz2) < unsigned(TZ);
            // the point's partial for this tile in its own slot (point-major layout), in the
            // arithmetic type: a wave sum of T values is exactly a T
            T* o = reinterpret_cast<T*>(out0) + ((long long)pk_point(ent) * G.maxp + pk_slot(ent)) * 3;
            // a tile of the point's window that holds no node of its stencil: its partial is zero
            if (!__any(in)) {
                if (lane == 0) o[0] = o[1] = o[2] = T(0);
                continue;
            }
            const int li = in ? lx2 + TX * (ly2 + TY * lz2) : 0;
            const T w = in ? r.wx[dx] * r.wy[dy] * r.wz[dz] : T(0);
            const T sx = wave_sum(su[0][li] * w);
            const T sy = wave_sum(su[1][li] * w);
            const T sz = wave_sum(su[2][li] * w);
            if (lane == 0) {
                o[0] = sx;
                o[1] = sy;
                o[2] = sz;
            }
        }
        if (G.tpb > 1) __syncthreads();   // su is rewritten by the block's next tile
    }
}

// Waves per SIMD the step kernel asks the compiler for (its register budget), where the
// default allocation would round up past a granule and lose a wave:
// - two FP16 nodes per lane, projected collision: this step waits mostly on memory and pays for
//   more waves than the 5 the compiler's 84 VGPRs allow unbounded: 7 (72 VGPRs, a few scalar
//   registers spilled to VGPR lanes) where a wave covers a tile row, 6 (80 VGPRs) for narrower
//   rows, whose per-lane neighbour loads need more registers;
// - one node per lane on tile rows of at least 64 nodes, FP32 arithmetic: the general collision
//   (7 waves, 72 VGPRs) and the thermal step (5 waves, 96 VGPRs), which would take 73-75 and
//   98-99 VGPRs unbounded.
// Only the two-node kernels on 128 x 1 x 2 and 256 x 1 x 1 tiles spill (one VGPR); the other
// forms (narrower rows, 64-bit addressing, FP64) would spill more and keep the default.
constexpr int step_waves(int ST, int TX, int NPL, int VAR, int COLL)
{
    if (VAR & 1) return 1;
    if (NPL == 2) return COLL == 0 ? (TX / NPL >= 64 ? 7 : 6) : 1;
    if ((ST == ST_FP32 || ST == ST_FP16) && TX >= 64) return COLL == 1 ? 7 : (COLL == 2 ? 5 : 1);
    return 1;
}

// One block per run of G.tpb consecutive tiles, in the block order G.order names
// (launch order, contiguous runs per XCD, or tile rows kept on one XCD); each tile is
// finished before the next.  BLOCK / NPL threads per block.  ONE (variant bit 128,
// with G.tpb == 1): the kernel is compiled for exactly one tile per block.  Without the
// tile loop the compiler has no loop to hoist the tile's wave-uniform values out of,
// values it otherwise keeps in scalar registers across the loop and spills into VGPR
// lanes (the thermal step: 47 such spills and 1111 VALU instructions with the loop,
// none and 864 without).  Both forms compute the same values bit for bit.
// With COLL == 2 the block of tile 0 also advances the step counter for the next
// step (*tout = *tin + 1; the two slots alternate with the population copies).
template <int ST, int TX, int TY, int TZ, int MODE, int VAR, int COLL = 0, int NPL = 1, bool ONE = false>
__global__ __launch_bounds__(BLOCK / NPL, MODE == M_STEP ? step_waves(ST, TX, NPL, VAR, COLL) : 1)
void k_lattice(const Geom G, const typename StoreT<ST>::S* __restrict__ src,
                                                   typename StoreT<ST>::S* __restrict__ dst,
                                                   const BoxDev* __restrict__ boxes, const int* __restrict__ toff,
                                                   const int* __restrict__ tlist,
                                                   const PRec<typename StoreT<ST>::T>* __restrict__ rec,
                                                   double* __restrict__ out0, double* __restrict__ out1,
                                                   const unsigned long long* __restrict__ tin,
                                                   unsigned long long* __restrict__ tout)
{
    const int b = int(blockIdx.x), nb = int(gridDim.x);
    const int first = (G.order == 1 ? b : G.order == 0 ? xcd_tile(b, nb) : row_group_run(b, nb, G.lgrp)) * G.tpb;
    if constexpr (ONE) {
        if (first < G.ntiles)
            lattice_tile<ST, TX, TY, TZ, MODE, VAR, COLL, NPL>(G, first, src, dst, boxes, toff, tlist, rec, out0, out1,
                                                               tin);
    } else {
        const int last = min((long long)first + G.tpb, G.ntiles);
        for (int tile = first; tile < last; ++tile)
            lattice_tile<ST, TX, TY, TZ, MODE, VAR, COLL, NPL>(G, tile, src, dst, boxes, toff, tlist, rec, out0, out1,
                                                               tin);
    }
    if constexpr (COLL == 2)
        if (first == 0 && threadIdx.x == 0) *tout = *tin + 1;
    // the tile lists of this step were current; the next step's records raise the flag again
    // if a point leaves its window
    if constexpr (MODE == M_STEP)
        if (first == 0 && threadIdx.x == 0) *G.rebin = 0;
}


// ---------------------------------------------------------------------------
// host-side launchers

// With ev0/ev1 set, the runtime stamps the two events at the kernel's own start
// and end (timing without the dispatch latency of separate event records).
template <int ST, int TX, int TY, int TZ, int VAR, int COLL, bool ONE>
static void launch_step_c(const Geom& G, const void* src, void* dst, BoxDev* boxes, const int* toff, const int* tlist,
                          const void* rec, double* out0, double* out1, const unsigned long long* tin,
                          unsigned long long* tout, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    using S = typename StoreT<ST>::S;
    using T = typename StoreT<ST>::T;
    const unsigned nb = (unsigned)((G.ntiles + G.tpb - 1) / G.tpb);
    if constexpr (ST == ST_FP16) {
        if (G.pairs) {
            // two nodes per lane
            if (ev0 && ev1)
                hipExtLaunchKernelGGL((k_lattice<ST, TX, TY, TZ, M_STEP, VAR, COLL, 2, ONE>), dim3(nb), dim3(BLOCK / 2), 0,
                                      s, ev0, ev1, 0, G, (const S*)src, (S*)dst, boxes, toff, tlist,
                                      (const PRec<T>*)rec, out0, out1, tin, tout);
            else
                hipLaunchKernelGGL((k_lattice<ST, TX, TY, TZ, M_STEP, VAR, COLL, 2, ONE>), dim3(nb), dim3(BLOCK / 2), 0, s,
                                   G, (const S*)src, (S*)dst, boxes, toff, tlist, (const PRec<T>*)rec, out0, out1, tin,
                                   tout);
            return;
        }
    }
    if (ev0 && ev1)
        hipExtLaunchKernelGGL((k_lattice<ST, TX, TY, TZ, M_STEP, VAR, COLL, 1, ONE>), dim3(nb), dim3(BLOCK), 0, s,
                              ev0, ev1, 0, G, (const S*)src, (S*)dst, boxes, toff, tlist, (const PRec<T>*)rec, out0,
                              out1, tin, tout);
    else
        hipLaunchKernelGGL((k_lattice<ST, TX, TY, TZ, M_STEP, VAR, COLL, 1, ONE>), dim3(nb), dim3(BLOCK), 0, s, G,
                           (const S*)src, (S*)dst, boxes, toff, tlist, (const PRec<T>*)rec, out0, out1, tin, tout);
}

template <int ST, int TX, int TY, int TZ, int VAR, bool ONE>
static void launch_step_v(const Geom& G, const void* src, void* dst, BoxDev* boxes, const int* toff, const int* tlist,
                          const void* rec, double* out0, double* out1, const unsigned long long* tin,
                          unsigned long long* tout, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1)
{
    // the general and thermal operators are instantiated with buffer addressing only (bit 0 off)
    if (G.coll == 2)
        launch_step_c<ST, TX, TY, TZ, VAR & ~1, 2, ONE>(G, src, dst, boxes, toff, tlist, rec, out0, out1, tin, tout, s, ev0,
                                                   ev1);
    else if (G.coll == 1)
        launch_step_c<ST, TX, TY, TZ, VAR & ~1, 1, ONE>(G, src, dst, boxes, toff, tlist, rec, out0, out1, tin, tout, s, ev0,
                                                   ev1);
    else
        launch_step_c<ST, TX, TY, TZ, VAR, 0, ONE>(G, src, dst, boxes, toff, tlist, rec, out0, out1, tin, tout, s, ev0, ev1);
}

template <int ST, int TX, int TY, int TZ, bool ONE>
static void launch_lattice_t(const Geom& G, int mode, int variant, const void* src, void* dst, BoxDev* boxes,
                             const int* toff, const int* tlist, const void* rec, double* out0, double* out1,
                             const unsigned long long* tin, unsigned long long* tout, hipStream_t s, hipEvent_t ev0,
                             hipEvent_t ev1)
{
    using S = typename StoreT<ST>::S;
    using T = typename StoreT<ST>::T;
    const unsigned nblocks = (unsigned)((G.ntiles + G.tpb - 1) / G.tpb);
    auto a0 = (const S*)src;
    auto a1 = (S*)dst;
    auto r = (const PRec<T>*)rec;
    if (mode == M_STEP) {
        switch (variant & 3) {
        case 1: launch_step_v<ST, TX, TY, TZ, 1, ONE>(G, src, dst, boxes, toff, tlist, rec, out0, out1, tin, tout, s, ev0, ev1); break;
        case 2: launch_step_v<ST, TX, TY, TZ, 2, ONE>(G, src, dst, boxes, toff, tlist, rec, out0, out1, tin, tout, s, ev0, ev1); break;
        case 3: launch_step_v<ST, TX, TY, TZ, 3, ONE>(G, src, dst, boxes, toff, tlist, rec, out0, out1, tin, tout, s, ev0, ev1); break;
        default: launch_step_v<ST, TX, TY, TZ, 0, ONE>(G, src, dst, boxes, toff, tlist, rec, out0, out1, tin, tout, s, ev0, ev1); break;
        }
    } else if constexpr (ONE) {
        // the one-tile instantiations are step kernels only
    } else if (mode == M_MOMENTS) {
        hipLaunchKernelGGL((k_lattice<ST, TX, TY, TZ, M_MOMENTS, 0>), dim3(nblocks), dim3(BLOCK), 0, s, G, a0, a1,
                           boxes, toff, tlist, r, out0, out1, nullptr, nullptr);
    } else {
        hipLaunchKernelGGL((k_lattice<ST, TX, TY, TZ, M_DIAG, 0>), dim3(nblocks), dim3(BLOCK), 0, s, G, a0, a1,
                           boxes, toff, tlist, r, out0, out1, nullptr, nullptr);
    }
}

template <int ST, bool ONE>
static bool launch_lattice_s(const Geom& G, int mode, int variant, const void* src, void* dst, BoxDev* boxes,
                             const int* toff, const int* tlist, const void* rec, double* out0, double* out1,
                             const unsigned long long* tin, unsigned long long* tout, hipStream_t s, hipEvent_t ev0,
                             hipEvent_t ev1)
{
#define LBM_TILE(X, Y, Z)                                                                                     \
    if (G.tx == X && G.ty == Y && G.tz == Z) {                                                                \
        launch_lattice_t<ST, X, Y, Z, ONE>(G, mode, variant, src, dst, boxes, toff, tlist, rec, out0, out1, tin, tout, s, \
                                      ev0, ev1);                                                              \
        return true;                                                                                          \
    }
    LBM_TILE(64, 2, 2)
    LBM_TILE(64, 4, 1)
    LBM_TILE(64, 1, 4)
    LBM_TILE(32, 4, 2)
    LBM_TILE(32, 2, 4)
    LBM_TILE(16, 4, 4)
    LBM_TILE(128, 2, 1)
    LBM_TILE(128, 1, 2)
    LBM_TILE(256, 1, 1)
#undef LBM_TILE
    return false;
}

}  // namespace lbm

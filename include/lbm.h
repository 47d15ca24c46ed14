/*
 * liblbm — forced D3Q19 lattice Boltzmann with off-lattice point forces on
 * MI355X (gfx950).  C ABI.
 *
 * Method: Nash, Adhikari & Cates, "Singular forces and point-like colloids in
 * lattice Boltzmann hydrodynamics".
 *   - Fluid step: the second-order forced LBE in auxiliary populations fbar
 *     (Sec. II, Eq. transformf and Eq. halftransform) with the projected-ghost
 *     MRT collision of Eq. fiexp: ghosts set to zero, all six stress modes
 *     relaxed at 1/tau, momentum A = sum fbar c + rho F, and stress
 *     B = S - omega (S - rho v v - tau (v F + F v)), omega = 1/(tau + 1/2)
 *     (the sign of the (S - rho v v) term is the one the general scheme
 *     Eq. mrtlbe implies).
 *   - Point forces: spread with Peskin's 4-point regularised delta,
 *     Eq. deltadef, F(r) = sum_a f_a deltaP(r - R_a) (Sec. III).
 *   - Fluid velocity at the particles: interpolated with the same kernel
 *     (Sec. IV), and colloids advanced by
 *     dR/dt = v(R) + F/(6 pi eta) (1/a - 1/a_L)   (Sec. IV).
 *
 * Conventions.  Lattice units dx = dt = 1.  Periodic boxes of nx*ny*nz nodes
 * at integer coordinates.  tau is the paper's relaxation time: the shear
 * viscosity is eta = rho0 tau / 3.  The grid field is the force density
 * g = rho F.  The physical velocity is u = (sum fbar c + g/2) / rho.
 * Populations are stored as deviations fbar_i - w_i rho0.
 *
 * Memory.  The caller owns all device memory: it allocates the workspace
 * (lb_workspace_bytes) and every input/output array, and must keep them alive
 * while work that uses them may still run.  The library allocates no device
 * memory.  Every call enqueues asynchronously on the stream given to lb_init
 * (or lb_set_stream) and returns without waiting, except lb_sync,
 * lb_diagnostics and lb_kernel_time, which wait for the stream.
 *
 * Errors.  Every int-returning call returns LB_OK (0) or a negative status;
 * lb_status_string() names it and lb_last_error() gives the context's last
 * message.  No exception crosses the ABI.  A device fault surfaces as
 * LB_ERR_HIP at the next call that checks the stream.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define LB_OK 0
#define LB_ERR_ARG (-1)       /* invalid argument */
#define LB_ERR_SIZE (-2)      /* workspace too small / size limits */
#define LB_ERR_HIP (-3)       /* HIP runtime error */
#define LB_ERR_NONFINITE (-4) /* non-finite value or FP16 overflow detected */
#define LB_ERR_CAPACITY (-5)  /* more point forces than max_points */
#define LB_ERR_STATE (-6)     /* call not valid in the current state */
#define LB_ERR_NEGATIVE_DENSITY (-7) /* a node's density rho0 + drho is <= 0 (lb_diagnostics) */

/* population storage */
#define LB_STORAGE_FP64 0 /* FP64 deviations, FP64 arithmetic */
#define LB_STORAGE_FP32 1 /* FP32 deviations, FP32 arithmetic */
#define LB_STORAGE_FP16 2 /* FP16 (fbar_i - w_i rho0)/w_i * 2^e per box, FP32 arithmetic */
#define LB_STORAGE_MOM32 3 /* FP32 post-collision moments, 10 per node instead of 19
                              populations (exact: with the ghosts projected out the
                              post-collision state of Eq. fiexp is fixed by rho, A, B);
                              FP32 arithmetic.  lb_set_equilibrium then sets the
                              equilibrium as the previous step's post-collision state. */

/* collision operators (lb_params.collision) */
#define LB_COLLISION_PROJECTED 0 /* Eq. fiexp: ghosts projected out, stress modes at 1/tau */
#define LB_COLLISION_BGK 1       /* Eq. bgklbe: every mode relaxes at 1/tau (ghosts kept) */
#define LB_COLLISION_MRT 2       /* Eq. mrtlbe with eigenvalues 1/tau on the five shear
                                    modes, 1/tau_bulk on the bulk mode and ghost_rate on
                                    all nine ghost modes */

/* point-force set kinds */
#define LB_FORCES_NEXT_STEP 0 /* applied in the next step only, then dropped */
#define LB_FORCES_STATIC 1    /* applied every step at fixed positions */
#define LB_COLLOIDS 2         /* applied every step; positions advanced in place */

#define LB_MAX_SETS 16
#define LB_NDIAG 13 /* values per box returned by lb_diagnostics */

/* MLP of the learned mobility correction: 4 -> 64 tanh -> 64 tanh -> 1 */
#define LBML_NPARAM 4545

typedef struct lb_params {
    int32_t nx, ny, nz;     /* nodes per box along x, y, z; each >= 4 */
    int32_t nboxes;         /* independent periodic boxes of that size, >= 1 */
    int32_t storage;        /* LB_STORAGE_* */
    int32_t zero_net_force; /* 1: add the uniform density -sum F / N per box */
    double rho0;            /* reference density (> 0); 0 means 1 */
    const double* tau;      /* HOST array [nboxes]: paper's tau (> 0) per box */
    int64_t max_points;     /* capacity: point forces over all sets at once; below 2^24
                               (LB_ERR_SIZE otherwise) */
    int32_t tile_x;         /* tile shape (nodes); 0 = default. tile_x*tile_y*tile_z = 256 */
    int32_t tile_y;
    int32_t tile_z;
    int32_t fp16_exponent;  /* FP16 only: initial scale exponent in [-100, 120] (the range the
                               exponent is kept in from step to step); 0 = default (30, or
                               from the thermal amplitude when kT > 0) */
    int32_t variant;        /* step-kernel variant bits (same results, different memory access):
                               1 = 64-bit per-lane addresses instead of scalar
                                   descriptors plus 32-bit lane offsets,
                               2 = cached instead of non-temporal population loads,
                               4 * k (k = 0..3) = each block of the step kernel works
                                   through 2^k consecutive tiles,
                               16 = blocks take tiles in launch order instead of
                                   contiguous runs of tiles per XCD,
                               32 = FP16 storage: one node per lane in the step
                                   kernel (by default, with nx even, each lane
                                   takes two adjacent x nodes with 32-bit
                                   accesses),
                               64 = the blocks of one tile row (all tiles with the
                                   same y, z tile index) run back to back on one
                                   XCD, tile rows in launch order across the XCDs
                                   (overrides 16; where the blocks per tile row are
                                   not a power of two, launch order),
                               128 = with one tile per block (4 * k = 0), a step
                                   kernel compiled for exactly one tile per block,
                                   without the tile loop: fewer scalar registers
                                   held and spilled (valid only with k = 0).
                               With LB_STORAGE_MOM32 bits 0 and 1 have no effect: each
                               node gathers the pieces of its 18 neighbours with cached
                               buffer loads. */
    int32_t collision;      /* LB_COLLISION_*; 0 = projected (the paper's operator) */
    const double* tau_bulk; /* LB_COLLISION_MRT: HOST array [nboxes] (> 0), read during
                               lb_init only; NULL = tau */
    double ghost_rate;      /* LB_COLLISION_MRT: eigenvalue of the ghost modes, in (0, 4];
                               a ghost moment is multiplied by (1 - r/2)/(1 + r/2) per
                               step; 2 projects them out.  LB_STORAGE_MOM32 keeps no
                               ghosts and accepts only collisions that project them out
                               (projected, or MRT with ghost_rate = 2). */
    double kT;              /* thermal energy (lattice units); 0 = deterministic.  > 0: the
                               fluctuating step (Sec. II): after the collision each
                               non-conserved mode k (bulk, five shear, nine ghost
                               polynomials of the orthogonal D3Q19 basis) receives a
                               Gaussian increment of variance (kT/cs^2) rho b_k
                               (1 - gamma_k^2), b_k its norm, gamma_k the factor the
                               collision applies to its non-equilibrium part (ghosts
                               therefore carry noise even when projected); LB_COLLOIDS
                               sets also receive the extra displacement of Appendix B,
                               variance kT/(3 pi eta)(1/a - 1/a_L) per step.  Not with
                               LB_STORAGE_MOM32. */
    uint64_t seed;          /* key of the Philox4x32-10 generator of the noise; the
                               draws of step t depend only on (seed, t, node or point
                               index), so a run is reproducible and independent of
                               tiles, variants, graphs and batching */
} lb_params;

/*
 * Per-set options for lb_add_point_forces.  For LB_COLLOIDS, inv_a = 1/a and
 * inv_aL = 1/a_L enter the update of Sec. IV; 1/a - 1/a_L must be > 0 (the
 * renormalised radius a_R is positive only for a < a_L).  If d_mlp is not
 * NULL, 1/a_L at each particle is inv_aL + out_scale * MLP(x) with
 * x_k = (raw_k - in_shift[k]) * in_scale[k] and raw = (frac(Rx), frac(Ry),
 * frac(Rz), tau of the particle's box); d_mlp holds LBML_NPARAM bfloat16
 * weights in the lbml layout.  d_vel_out (n,3) FP64 receives the interpolated
 * fluid velocity v(R) of the last step; d_vel_sum (n,3) FP64 is incremented by
 * it every step (the caller zeroes it).  Either may be NULL.
 */
typedef struct lb_point_model {
    double inv_a;
    double inv_aL;
    const uint16_t* d_mlp;
    float in_shift[4];
    float in_scale[4];
    float out_scale;
    double* d_vel_out;
    double* d_vel_sum;
} lb_point_model;

typedef struct lb_ctx lb_ctx;

/* Device bytes the workspace must have for these parameters.  Pure function. */
int lb_workspace_bytes(const lb_params* p, size_t* bytes);

/*
 * Create a context on the caller's workspace (device pointer, >= the queried
 * size, 256-byte aligned) and set every box to rest (fbar = w rho0, i.e. zero
 * deviation).  hip_stream is a hipStream_t (NULL = the null stream).  The
 * context holds, but does not own, the workspace.
 */
int lb_init(const lb_params* p, void* d_workspace, size_t bytes, void* hip_stream, lb_ctx** out);

/* Redirect subsequent work to another stream. */
int lb_set_stream(lb_ctx* ctx, void* hip_stream);

/*
 * Set the auxiliary populations of every node to the equilibrium of Eq. eqf at
 * the given density and velocity: d_rho (nboxes,nz,ny,nx) and d_u
 * (nboxes,3,nz,ny,nx), FP64 device arrays.
 */
int lb_set_equilibrium(lb_ctx* ctx, const double* d_rho, const double* d_u);

/*
 * Register n point forces: d_pos and d_force are (n,3) FP64 device arrays,
 * positions in lattice units (wrapped periodically), forces in lattice units
 * (force per step).  d_box (n) int32 names each point's box, or NULL for box 0.
 * kind is one of the LB_FORCES_ kinds or LB_COLLOIDS; model may be NULL except for colloids.
 * LB_FORCES_NEXT_STEP and LB_COLLOIDS arrays are read at every step that
 * applies them; LB_FORCES_STATIC arrays are read once, before the first step
 * after registration (re-register to change them).  All must stay valid until
 * the work that reads them has run (stream order).  Positions and box ids of the
 * sets read every step may be rewritten between steps by any amount: each point
 * is binned to the tiles of a 5-node window per axis around its stencil, and
 * the tile lists are rebuilt in the step at which a stencil has left its window
 * (or its box changed), choosing new windows for the points of that box only.  Forces spread per
 * Sec. III; multipoles are passed as their point forces (see
 * lb_expand_multipoles).  With FP16 storage the scale exponent follows the
 * data with one step of delay: a jump of more than 4x in the largest
 * population deviation within one step overflows and is reported as
 * LB_ERR_NONFINITE.
 */
int lb_add_point_forces(lb_ctx* ctx, int64_t n, const double* d_pos, const double* d_force,
                        const int32_t* d_box, int kind, const lb_point_model* model);

/*
 * Singular forces on curves and surfaces (Sec. I; Eq. singularF with a line or
 * area measure), carried by markers that move with the fluid.  The library
 * computes each marker's force from the set's configuration at every step,
 * writes it to d_force, spreads it like a point force (Sec. III), interpolates
 * the velocity U at the marker (Sec. IV) and moves the marker by R <- R + U
 * (no point-particle mobility terms, no thermal displacement).
 *
 * LB_ELASTIC_CHAIN: markers form consecutive chains of chain_len (>= 2, n a
 *   multiple of it); markers i and i+1 of one chain are joined by a Hookean
 *   spring, force k_spring (|d| - l0) d/|d| on i and its opposite on i+1,
 *   d = R_{i+1} - R_i taken as the nearest periodic image.
 * LB_ELASTIC_SURFACE: a closed triangulated surface of tension `tension`;
 *   vertex force -tension dA/dR_v, where for a triangle (a, b, c) ordered
 *   counter-clockwise about its unit normal n, dA/da = n x (c - b) / 2.
 *   d_tri (ntri,3) vertex indices; the incidence d_vt_off (n+1) / d_vt_idx
 *   (3 ntri) lists, per vertex, the triangles containing it (CSR, ascending).
 * Both: optional external force per marker d_ext (n,3) added to the elastic
 * force; d_box (n) the box of each marker or NULL (box 0), one set in one box.
 * Arrays are FP64 / int32 device arrays owned by the caller and must stay valid
 * while the set is registered; d_pos is updated in place, d_force overwritten.
 * Errors: LB_ERR_ARG (bad kind, sizes, NULL arrays, non-finite parameters),
 * LB_ERR_CAPACITY (markers beyond max_points together with the other sets).
 */
#define LB_ELASTIC_CHAIN 0
#define LB_ELASTIC_SURFACE 1

typedef struct lb_elastic {
    int32_t kind;            /* LB_ELASTIC_CHAIN or LB_ELASTIC_SURFACE */
    int32_t chain_len;       /* chain: markers per chain */
    int64_t n;               /* markers */
    double* d_pos;           /* (n,3) positions, advanced in place */
    double* d_force;         /* (n,3) written each step with the marker forces */
    const double* d_ext;     /* (n,3) external forces or NULL */
    const int32_t* d_box;    /* (n) box ids or NULL */
    double* d_vel_out;       /* (n,3) interpolated velocity of the last step, or NULL */
    double k_spring, l0;     /* chain */
    double tension;          /* surface */
    int64_t ntri;            /* surface */
    const int32_t* d_tri;    /* surface: (ntri,3) */
    const int32_t* d_vt_off; /* surface: (n+1) */
    const int32_t* d_vt_idx; /* surface: (3 ntri) */
} lb_elastic;

int lb_add_elastic(lb_ctx* ctx, const lb_elastic* set);

/* Drop every registered set. */
int lb_clear_forces(lb_ctx* ctx);

/*
 * Advance nsteps steps.  Each step: spread the registered forces at the
 * current positions, collide every node with them (Eq. fiexp), interpolate the
 * physical velocity u at the points with the same kernel, propagate (the split
 * after Eq. halftransform), then advance colloids by the Sec. IV update
 * (explicit Euler).  Repeated chunks of 2, 4, ..., 128 steps run as captured
 * HIP graphs (captured on first use per chunk length, parity and set of
 * registered forces).  Returns after enqueueing.  Conditions the kernels flag
 * (LB_ERR_NONFINITE for a non-finite value or FP16 overflow, LB_ERR_ARG for a
 * box id out of range, LB_ERR_STATE when a tile-list rebuild's device-wide
 * barrier wait ran out) are reported by the next call that reads the flags
 * (lb_sync, lb_diagnostics).
 */
int lb_step(lb_ctx* ctx, int32_t nsteps);

/*
 * Capture, without running them, the HIP graphs that lb_step(ctx, nsteps) would
 * replay from the current state (registered sets, population parity), so that a
 * caller who times lb_step keeps graph capture out of the timed region.  No step
 * is taken and nothing is enqueued; the state is unchanged.  With a pending
 * next-step set, in timing mode or for nsteps < 4 there is nothing to capture
 * ahead (LB_OK).  Errors: LB_ERR_ARG (ctx NULL, nsteps < 0), LB_ERR_HIP (capture
 * failed).
 */
int lb_prepare_steps(lb_ctx* ctx, int32_t nsteps);

/*
 * Physical moments at the current time with the registered forces
 * (Eq. macrovariables2): d_rho (nboxes,nz,ny,nx), d_u (nboxes,3,nz,ny,nx),
 * FP64 device arrays; d_rho may be NULL.
 */
int lb_moments(lb_ctx* ctx, double* d_rho, double* d_u);

/*
 * Interpolated physical velocity U(R) = sum_x u(x) deltaP(x - R) (Sec. IV) at
 * n arbitrary points: d_pos (n,3) FP64, d_box (n) int32 or NULL, d_u_out (n,3).
 */
int lb_interp_velocity(lb_ctx* ctx, int64_t n, const double* d_pos, const int32_t* d_box, double* d_u_out);

/*
 * FP64 diagnostics per box, written to HOST h_out[nboxes][LB_NDIAG]:
 *   0 sum drho, 1-3 sum jbar (auxiliary momentum), 4-6 sum g,
 *   7-9 sum x cross g (node coordinates in the box), 10 max |u|,
 *   11 count of non-finite nodes, 12 count of nodes whose density
 *   rho0 + drho is not positive (finite nodes only).  Waits for the stream.
 *   Returns LB_ERR_NONFINITE if any box holds a non-finite value, else
 *   LB_ERR_NEGATIVE_DENSITY if any node has a non-positive density (the
 *   lattice has left the physical range: Ma too large for the forcing);
 *   h_out is written in both cases.
 */
int lb_diagnostics(lb_ctx* ctx, double* h_out);

/* Wait for the stream; reports a pending device error or non-finite flag. */
int lb_sync(lb_ctx* ctx);

/*
 * Checkpoint and resume.  The state of a context between steps - the current
 * populations, the per-box records (FP16 exponents, counter-force), the FP16
 * tile maxima, the thermal step counter, the non-finite flags and the binning
 * windows of the points - is copied to or from a caller buffer (device or
 * pinned host memory, 256-byte aligned, at least lb_checkpoint_bytes bytes;
 * the copies are stream-ordered).  Point positions and forces stay the
 * caller's arrays: save them alongside.  To resume, create a context with the
 * same lb_params, register the same sets (same kinds, sizes and order, the
 * saved positions) and call lb_checkpoint_load before stepping: the resumed
 * run then continues bit for bit as the uninterrupted run would.
 * lb_checkpoint_save needs the registered points to have been binned (a step,
 * or lb_moments, since the sets last changed): LB_ERR_STATE otherwise.
 * lb_checkpoint_load waits for the stream, checks the saved header against
 * the context (LB_ERR_ARG on a mismatch) and sets lb_steps_taken to the saved
 * count.
 */
int lb_checkpoint_bytes(const lb_ctx* ctx, size_t* bytes);
int lb_checkpoint_save(lb_ctx* ctx, void* d_dst);
int lb_checkpoint_load(lb_ctx* ctx, const void* d_src);

/* Release the context (host memory and cached graphs); the workspace stays the caller's. */
int lb_destroy(lb_ctx* ctx);

const char* lb_status_string(int status);
const char* lb_last_error(const lb_ctx* ctx);

/* Steps taken since lb_init. */
int64_t lb_steps_taken(const lb_ctx* ctx);

/*
 * Timing of the fused step kernel: with enable = 1, lb_step launches eagerly
 * and every fused-kernel launch carries a pair of HIP events that the runtime
 * stamps at the kernel's own start and end on the context's stream;
 * lb_kernel_time waits for the stream and returns the summed duration (ms)
 * and the number of launches since timing was enabled.
 */
int lb_kernel_timing(lb_ctx* ctx, int enable);
int lb_kernel_time(lb_ctx* ctx, double* total_ms, int64_t* launches);

/*
 * Streaming-copy probe (a measurement aid, not an operation of the method):
 * copies `bytes` from d_src to d_dst (device pointers, both 16-byte aligned,
 * non-overlapping, bytes a positive multiple of 16), 16 bytes per thread with
 * non-temporal loads and stores, enqueued on hip_stream (NULL = default
 * stream).  Timed by the caller, it gives the practical HBM copy rate against
 * which the fused step kernel's bandwidth is set beside the vendor peak.
 * Errors: LB_ERR_ARG (alignment, size, overlap), LB_ERR_SIZE (grid too large),
 * LB_ERR_HIP (launch failure).
 */
int lb_copy_probe(const void* d_src, void* d_dst, size_t bytes, void* hip_stream);

/*
 * Multipoles of Sec. III as point forces (HOST arrays, host computation).
 * type[i]: 0 Stokeslet (s p at R), 1 stresslet (+s p at R + d/2 p and
 * -s p at R - d/2 p), 2 rotlet (with e2 = n x e1: +s e2 at R + d/2 e1,
 * -s e2 at R - d/2 e1, -s e1 at R + d/2 e2, +s e1 at R - d/2 e2: zero net
 * force, zero symmetric part, torque 2 d s n).  axis is p (types 0, 1) or
 * n (type 2), unit; e1 is a unit vector normal to n.  Outputs hold up to
 * 4 n points; *n_out receives the count.  Points keep the input order.
 */
int lb_expand_multipoles(int64_t n, const int32_t* type, const double* center, const double* axis,
                         const double* e1, const double* strength, double sep, int64_t* n_out,
                         double* pos_out, double* force_out);

/*
 * Mobility-correction MLP (not in the paper: it predicts the
 * lattice-position dependence of 1/a_L defined in Sec. IV / Appendix A).
 * Parameter layout (flat): W1[64][4], b1[64], W2[64][64], b2[64], W3[1][64], b3[1].
 * Device arrays; stream-ordered on hip_stream.
 *   lbml_round_bf16: w16[i] = bf16(master[i]) (round to nearest even).
 *   lbml_forward:    y[n] = MLP(x[n][4]) with bf16 weights, FP32 accumulation.
 *   lbml_loss_grad:  grad[LBML_NPARAM] (FP32) = d/dtheta mean((y - target)^2)
 *                    at the bf16 weights, and *loss (FP32 device scalar);
 *                    deterministic (fixed reduction order).  work must hold
 *                    lbml_work_floats(n) floats.
 *   lbml_adam_step:  one Adam update (Kingma & Ba) of master/m/v at iteration t
 *                    and re-rounding of w16.
 */
int64_t lbml_work_floats(int64_t n);
int lbml_round_bf16(const float* d_master, uint16_t* d_w16, void* hip_stream);
int lbml_forward(const uint16_t* d_w16, int64_t n, const float* d_x, float* d_y, void* hip_stream);
int lbml_loss_grad(const uint16_t* d_w16, int64_t n, const float* d_x, const float* d_target, float* d_grad,
                   float* d_loss, float* d_work, void* hip_stream);
int lbml_adam_step(float* d_master, float* d_m, float* d_v, const float* d_grad, uint16_t* d_w16, int32_t t,
                   float lr, float beta1, float beta2, float eps, void* hip_stream);

/*
 * lbml_loss_grad without a work argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving or training
 * loops, harnesses that forbid allocation): the per-sample work lives in a
 * device array inside the library, sized for n <= LBML_STATIC_MAX_N samples
 * (4.2 MB, held on each device the library runs on until the process ends).
 * Same results as lbml_loss_grad, bit for bit.  The call allocates nothing;
 * its first call on a device looks up that device's copy of the array.
 * Errors: LB_ERR_ARG (n <= 0, NULL pointers), LB_ERR_SIZE (n above
 * LBML_STATIC_MAX_N), LB_ERR_HIP.  Every call on one device uses the same
 * array: calls that may overlap on one device (other streams, other threads)
 * race and must be ordered by the caller.
 */
#define LBML_STATIC_MAX_N 4096
int lbml_loss_grad_static(const uint16_t* d_w16, int64_t n, const float* d_x, const float* d_target, float* d_grad,
                          float* d_loss, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */

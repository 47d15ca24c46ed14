// liblbm host runtime: the C ABI declared in include/lbm.h.
//
// The context owns no device memory: it carves the caller's workspace into
// the two population copies (pull scheme, A/B), per-box parameters, the
// per-point records, the tile bins and the scratch of the reductions, and
// enqueues every kernel on the caller's stream.  Repeated steps are captured
// once per (parity, force-set generation, length) into HIP graphs of 2, 4,
// ..., 128 steps and replayed.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_device.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

constexpr size_t ALIGN = 256;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// Multiplier and shift for n / d with n < 2^31 (d >= 1): s = 31 + ceil(log2 d), m = ceil(2^s / d)
// (below 2^32 for every d >= 1); then n / d = (n * m) >> s exactly.
void set_div_magic(int d, unsigned& m, int& s)
{
    int l = 0;
    while ((1LL << l) < d) ++l;
    s = 31 + l;
    m = unsigned(((1ULL << s) + (unsigned long long)d - 1) / (unsigned long long)d);
}

size_t storage_bytes(int st) { return st == LB_STORAGE_FP64 ? 8 : (st == LB_STORAGE_FP16 ? 2 : 4); }

size_t rec_bytes(int st) { return st == LB_STORAGE_FP64 ? sizeof(PRec<double>) : sizeof(PRec<float>); }

// most tiles of extent t met by the binning window of a point (5 consecutive nodes, periodic)
int max_axis_tiles(int n, int t)
{
    constexpr int WIN = 5;
    int best = 0;
    for (int b = 0; b < n; ++b) {
        int seen[WIN], cnt = 0;
        for (int k = 0; k < WIN; ++k) {
            const int tile = ((b + k) % n) / t;
            bool dup = false;
            for (int j = 0; j < cnt; ++j) dup |= seen[j] == tile;
            if (!dup) seen[cnt++] = tile;
        }
        best = std::max(best, cnt);
    }
    return best;
}

struct Layout {
    size_t pop[2], boxes, rec, psum, count, cursor, toff, bsum, tlist, tlist_tmp, partial, fpart, pmax, tmax, smax, ticket,
        tctr,
        err, nf, rebin, rebox, win,
        diag, diagout;
    size_t total;
};

struct Plan {
    Geom G;
    Layout L;
    int chunks;
    long long cap;
};

void choose_tile(const lb_params* p, int& tx, int& ty, int& tz)
{
    if (p->tile_x > 0) {
        tx = p->tile_x;
        ty = p->tile_y;
        tz = p->tile_z;
        return;
    }
    const double box_bytes = double(p->nx) * p->ny * p->nz * planes_of(p->storage) * storage_bytes(p->storage);
    if (p->storage == LB_STORAGE_MOM32 && p->nx >= 128) {
        tx = 128; ty = 1; tz = 2;   // long x rows: the gathered pieces are re-read from L1
    } else if (box_bytes >= 4.0e9) {
        tx = 128; ty = 2; tz = 1;   // a whole wave on one row (also with two FP16 nodes per lane)
    } else if (p->nx >= 64) {
        tx = 64; ty = 2; tz = 2;
    } else if (p->nx >= 32) {
        tx = 32; ty = 4; tz = 2;
    } else {
        tx = 16; ty = 4; tz = 4;
    }
}

int make_plan(const lb_params* p, Plan& P, std::string& why)
{
    if (!p) { why = "params is NULL"; return LB_ERR_ARG; }
    if (p->nx < 4 || p->ny < 4 || p->nz < 4) { why = "each of nx, ny, nz must be >= 4"; return LB_ERR_ARG; }
    if (p->nboxes < 1) { why = "nboxes must be >= 1"; return LB_ERR_ARG; }
    if (p->storage < LB_STORAGE_FP64 || p->storage > LB_STORAGE_MOM32) { why = "unknown storage"; return LB_ERR_ARG; }
    if (p->max_points < 0) { why = "max_points must be >= 0"; return LB_ERR_ARG; }
    if (!(p->rho0 >= 0.0) || !isfinite(p->rho0)) { why = "rho0 must be finite and >= 0"; return LB_ERR_ARG; }
    if (p->variant < 0 || p->variant > 255) { why = "unknown kernel variant"; return LB_ERR_ARG; }
    if ((p->variant & 128) && ((p->variant >> 2) & 3)) { why = "variant 128 needs one tile per block"; return LB_ERR_ARG; }
    if (p->collision < LB_COLLISION_PROJECTED || p->collision > LB_COLLISION_MRT) {
        why = "unknown collision operator";
        return LB_ERR_ARG;
    }
    if (p->collision == LB_COLLISION_MRT && !(p->ghost_rate > 0.0 && p->ghost_rate <= 4.0)) {
        why = "ghost_rate must be in (0, 4]";
        return LB_ERR_ARG;
    }
    if (p->storage == LB_STORAGE_MOM32 &&
        (p->collision == LB_COLLISION_BGK || (p->collision == LB_COLLISION_MRT && p->ghost_rate != 2.0))) {
        why = "moment storage keeps no ghost moments: the collision must project them out";
        return LB_ERR_ARG;
    }
    if (!(p->kT >= 0.0) || !isfinite(p->kT)) { why = "kT must be finite and >= 0"; return LB_ERR_ARG; }
    if (p->fp16_exponent < -100 || p->fp16_exponent > 120) {
        why = "fp16_exponent must lie in [-100, 120] (the range the scale exponent is kept in)";
        return LB_ERR_ARG;
    }
    if (p->storage == LB_STORAGE_MOM32 && p->kT > 0.0) {
        why = "moment storage keeps no ghost moments: thermal noise needs population storage";
        return LB_ERR_ARG;
    }
    int tx, ty, tz;
    choose_tile(p, tx, ty, tz);
    if (!tile_supported(tx, ty, tz)) { why = "unsupported tile shape"; return LB_ERR_ARG; }
    Geom& G = P.G;
    memset(&G, 0, sizeof(G));
    G.nx = p->nx; G.ny = p->ny; G.nz = p->nz; G.nboxes = p->nboxes;
    G.tx = tx; G.ty = ty; G.tz = tz;
    G.ltx = __builtin_ctz(tx); G.lty = __builtin_ctz(ty); G.ltz = __builtin_ctz(tz);
    G.ntx = (p->nx + tx - 1) / tx;
    G.nty = (p->ny + ty - 1) / ty;
    G.ntz = (p->nz + tz - 1) / tz;
    set_div_magic(G.ntx, G.mtx, G.stx);
    set_div_magic(G.nty, G.mty, G.sty);
    set_div_magic(G.ntz, G.mtz, G.stz);
    G.N = (long long)p->nx * p->ny * p->nz;
    G.kp = p->nx;
    G.rb = (long long)planes_of(p->storage) * p->nx;
    G.sbox = ((long long)p->ny * p->nz * G.rb + 255) / 256 * 256 + 64;
    {
        // lanes along x of one tile row: a wave on one row addresses each row block from
        // its own descriptor; narrower rows of lanes address the box from one descriptor
        // with 32-bit offsets
        const bool pairs = p->storage == LB_STORAGE_FP16 && p->nx % 2 == 0 && !((p->variant >> 5) & 1);
        const int lanes_x = pairs ? tx / 2 : tx;
        if (lanes_x < 64 && (unsigned long long)G.sbox * storage_bytes(p->storage) >= (1ULL << 32)) {
            why = "tiles with fewer than 64 lanes along x (64 nodes, or 128 with two FP16 nodes per lane) need a "
                  "box of under 4 GiB";
            return LB_ERR_ARG;
        }
        // two FP16 nodes per lane on whole-wave rows address each z plane of rows from one descriptor
        if (pairs && lanes_x >= 64 && (unsigned long long)p->ny * G.rb * storage_bytes(p->storage) >= (1ULL << 32)) {
            why = "two FP16 nodes per lane need a z plane (ny * nx nodes) of under 4 GiB";
            return LB_ERR_SIZE;
        }
    }
    G.tiles_per_box = (long long)G.ntx * G.nty * G.ntz;
    G.ntiles = G.tiles_per_box * p->nboxes;
    G.rho0 = p->rho0 > 0.0 ? p->rho0 : 1.0;
    G.maxp = max_axis_tiles(p->nx, tx) * max_axis_tiles(p->ny, ty) * max_axis_tiles(p->nz, tz);
    if (G.ntiles >= (1LL << 31) - 1) { why = "too many tiles"; return LB_ERR_SIZE; }
    P.cap = p->max_points;
    if (P.cap * G.maxp >= (1LL << 31) - 1 || P.cap >= (1LL << (31 - PK_SHIFT))) {
        why = "max_points too large";
        return LB_ERR_SIZE;
    }
    if (G.maxp > (1 << PK_BITS)) { why = "tile too small for the stencil"; return LB_ERR_ARG; }
    G.bchunks = int(std::min<long long>(256, (G.tiles_per_box + 255) / 256));
    G.tpb = 1 << ((p->variant >> 2) & 3);
    G.order = (p->variant >> 4) & 1;
    G.lgrp = 0;
    if ((p->variant >> 6) & 1) {
        // the runs of one tile row on one XCD: needs a power-of-two count of whole runs per row
        // (otherwise launch order)
        G.order = 1;
        if (G.ntx % G.tpb == 0 && ((G.ntx / G.tpb) & (G.ntx / G.tpb - 1)) == 0) {
            G.order = 2;
            G.lgrp = __builtin_ctz(unsigned(G.ntx / G.tpb));
        }
    }
    G.pairs = p->storage == LB_STORAGE_FP16 && p->nx % 2 == 0 && !((p->variant >> 5) & 1);
    G.coll = p->kT > 0.0 ? 2 : (p->collision != LB_COLLISION_PROJECTED ? 1 : 0);
    G.seed_lo = uint32_t(p->seed);
    G.seed_hi = uint32_t(p->seed >> 32);
    G.one = 1.0f;
    P.chunks = G.bchunks;
    Layout& L = P.L;
    size_t o = 0;
    auto take = [&](size_t bytes) { const size_t at = o; o = align_up(o + std::max<size_t>(bytes, 1)); return at; };
    const size_t popb = (size_t)G.sbox * p->nboxes * storage_bytes(p->storage);
    L.pop[0] = take(popb);
    L.pop[1] = take(popb);
    L.boxes = take(sizeof(BoxDev) * p->nboxes);
    L.rec = take(rec_bytes(p->storage) * P.cap);
    L.psum = take(sizeof(double) * 3 * (prep_blocks(P.cap) + LB_MAX_SETS));
    L.count = take(sizeof(int) * G.ntiles);
    L.cursor = take(sizeof(int) * G.ntiles);
    L.toff = take(sizeof(int) * (G.ntiles + 1));
    L.bsum = take(sizeof(int) * scan_blocks(G.ntiles));
    L.tlist = take(sizeof(int) * P.cap * G.maxp);
    L.tlist_tmp = take(sizeof(int) * P.cap * G.maxp);
    L.partial = take(sizeof(double) * 3 * P.cap * G.maxp);
    L.fpart = take(sizeof(double) * 3 * p->nboxes * P.chunks);
    L.pmax = take(sizeof(float) * p->nboxes * P.chunks);
    L.tmax = take(sizeof(float) * G.ntiles);
    L.smax = take(sizeof(unsigned) * SMAX_SLOTS * SMAX_STRIDE);
    L.ticket = take(sizeof(unsigned) * p->nboxes);
    L.tctr = take(2 * sizeof(unsigned long long));
    L.err = take(sizeof(int) * 4);
    L.nf = take(sizeof(int) * p->nboxes);
    L.rebin = take(sizeof(int));
    L.rebox = take(sizeof(int) * p->nboxes);
    L.win = take(sizeof(int4) * P.cap);
    L.diag = take(sizeof(double) * LBD_N * G.ntiles);
    L.diagout = take(sizeof(double) * LBD_N * p->nboxes);
    L.total = o;
    return LB_OK;
}

// set kind of marker sets (curves and surfaces); the public kinds are 0..2
constexpr int KIND_ELASTIC = 100;

struct Set {
    long long n;
    const double* pos;
    const double* frc;
    const int* box;
    int kind;
    lb_point_model model;
    bool has_model;
    lb_elastic el;   // KIND_ELASTIC only
};

// longest captured chunk of steps (a power of two; graphs of 2, 4, ..., GRAPH_MAX steps)
constexpr int GRAPH_MAX = 128;

// Header of a checkpoint (see lb_checkpoint_save): what the state was taken from, and where each
// section starts in the blob.
struct CkptHeader {
    char magic[8];
    int32_t nx, ny, nz, nboxes, storage, collision, tx, ty, tz, pad;
    int64_t steps, npoints, pop_bytes, tiles, total;
    int64_t off_pop, off_boxes, off_tmax, off_smax, off_tctr, off_nf, off_win;
};
constexpr char CKPT_MAGIC[8] = {'l', 'b', 'c', 'k', 'p', 't', '0', '1'};

struct GraphEntry {
    int parity;
    unsigned long long gen;
    int len;
    hipGraph_t graph;
    hipGraphExec_t exec;
};

}  // namespace

struct lb_ctx {
    lb_params p;
    std::vector<double> tau;
    Plan P;
    char* ws;
    hipStream_t stream;
    hipStream_t cap_stream;
    int cur;
    std::vector<Set> sets;
    unsigned long long gen;
    unsigned long long binned_gen;   // gen the tile lists were last forced to rebuild for
    bool bins_valid;
    bool gc_valid;   // counter-force sums current for the registered static sets
    std::vector<GraphEntry> graphs;
    bool timing;
    std::vector<hipEvent_t> ev;
    size_t ev_used;
    double timed_ms;
    long long timed_launches;
    long long steps;
    CkptHeader ckpt;   // header of the last checkpoint taken (read by its stream-ordered copy)
    std::vector<BoxDev> hboxes;
    std::string err;

    void* pop(int k) const { return ws + P.L.pop[k]; }
    BoxDev* boxes() const { return (BoxDev*)(ws + P.L.boxes); }
    void* rec() const { return ws + P.L.rec; }
    double* psum() const { return (double*)(ws + P.L.psum); }
    int* count() const { return (int*)(ws + P.L.count); }
    int* cursor() const { return (int*)(ws + P.L.cursor); }
    int* toff() const { return (int*)(ws + P.L.toff); }
    int* bsum() const { return (int*)(ws + P.L.bsum); }
    int* tlist() const { return (int*)(ws + P.L.tlist); }
    int* tlist_tmp() const { return (int*)(ws + P.L.tlist_tmp); }
    double* partial() const { return (double*)(ws + P.L.partial); }
    double* fpart() const { return (double*)(ws + P.L.fpart); }
    float* pmax() const { return (float*)(ws + P.L.pmax); }
    float* tmax() const { return (float*)(ws + P.L.tmax); }
    unsigned* smax() const { return (unsigned*)(ws + P.L.smax); }
    unsigned* ticket() const { return (unsigned*)(ws + P.L.ticket); }
    unsigned long long* tctr() const { return (unsigned long long*)(ws + P.L.tctr); }
    int* errw() const { return (int*)(ws + P.L.err); }
    int* nf() const { return (int*)(ws + P.L.nf); }
    int* rebin() const { return (int*)(ws + P.L.rebin); }
    int* rebox() const { return (int*)(ws + P.L.rebox); }
    int4* win() const { return (int4*)(ws + P.L.win); }
    double* diag() const { return (double*)(ws + P.L.diag); }
    double* diagout() const { return (double*)(ws + P.L.diagout); }
};

namespace {

thread_local std::string g_err;  // message of the last failure without a context

int fail(lb_ctx* c, int code, const std::string& msg)
{
    if (c)
        c->err = msg;
    else
        g_err = msg;
    return code;
}

// Launch errors are read with hipGetLastError after our own launches; drop
// any error an earlier, unrelated runtime call left behind first.
void clear_stale_error() { (void)hipGetLastError(); }

int hip_check(lb_ctx* c, hipError_t e, const char* what)
{
    if (e == hipSuccess) return LB_OK;
    return fail(c, LB_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

long long total_points(const lb_ctx* c)
{
    long long n = 0;
    for (auto& s : c->sets) n += s.n;
    return n;
}

bool has_kind(const lb_ctx* c, int kind)
{
    for (auto& s : c->sets)
        if (s.kind == kind) return true;
    return false;
}

// After the sets change, the next list build must run whatever the positions:
// raise the rebuild flag once per change.  Enqueued eagerly, never into a
// captured graph (a graph replays every node it holds).
void force_rebin(lb_ctx* c, hipStream_t s)
{
    if (c->binned_gen == c->gen) return;
    launch_fill_u32(c->rebin(), 1, 1u, s);
    launch_fill_u32(c->rebox(), c->p.nboxes, 1u, s);
    c->binned_gen = c->gen;
}

// blocks of point-force sums the records kernel writes (one box only; see k_prep)
long long npsum(const lb_ctx* c)
{
    long long nb = 0;
    for (auto& s : c->sets) nb += prep_blocks(s.n);
    return nb;
}

// records + tile bins for the current point positions (the binning kernels
// rebuild the lists only while the rebuild flag is set)
void build_points(lb_ctx* c, hipStream_t s)
{
    const Geom& G = c->P.G;
    long long off = 0, blk = 0;
    for (auto& st : c->sets) {
        double* ps = G.nboxes == 1 ? c->psum() + 3 * blk : nullptr;
        launch_prep(c->p.storage, G, st.n, off, st.pos, st.frc, st.box, c->rec(), c->errw(), ps, s);
        off += st.n;
        blk += prep_blocks(st.n);
    }
    launch_bins(c->p.storage, G, off, c->rec(), c->count(), c->bsum(), c->toff(), c->cursor(), c->tlist(),
                c->tlist_tmp(), c->errw(), s);
    c->gc_valid = false;
}

// per-box work before a step or a read: the counter-force sums (only when the
// point records may have changed since they were last taken) and the FP16
// exponent of the coming step
void box_update(lb_ctx* c, hipStream_t s, bool fp16_exp)
{
    const bool sums = c->p.zero_net_force != 0 && !c->gc_valid;
    const bool fp16 = fp16_exp && c->p.storage == LB_STORAGE_FP16;
    if (!sums && !fp16) return;
    const bool one = c->P.G.nboxes == 1;
    launch_box_update(c->p.storage, c->P.G, c->rec(), total_points(c) > 0 ? c->toff() : nullptr, c->tlist(),
                      one ? c->psum() : nullptr, one ? npsum(c) : 0, c->tmax(), c->fpart(), c->pmax(), c->ticket(),
                      c->boxes(), sums ? 1 : 0, fp16 ? 1 : 0, s);
    if (sums) c->gc_valid = true;
}

// marker forces of the curve and surface sets from their current configuration
void elastic_forces(lb_ctx* c, hipStream_t s)
{
    const Geom& G = c->P.G;
    for (auto& st : c->sets)
        if (st.kind == KIND_ELASTIC) {
            ElasticLaunch e;
            e.kind = st.el.kind;
            e.chain_len = st.el.chain_len;
            e.n = st.n;
            e.pos = st.pos;
            e.ext = st.el.d_ext;
            e.frc = st.el.d_force;
            e.k_spring = st.el.k_spring;
            e.l0 = st.el.l0;
            e.tension = st.el.tension;
            e.tri = st.el.d_tri;
            e.vt_off = st.el.d_vt_off;
            e.vt_idx = st.el.d_vt_idx;
            launch_elastic_forces(G, e, s);
        }
}

// one step on stream s; flips c->cur
void enqueue_step(lb_ctx* c, hipStream_t s, bool rebuild)
{
    const Geom& G = c->P.G;
    const long long npts = total_points(c);
    elastic_forces(c, s);
    if (npts > 0 && rebuild) build_points(c, s);
    box_update(c, s, true);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        if (c->ev_used + 2 > c->ev.size()) {
            for (int k = 0; k < 256; ++k) {
                hipEvent_t e;
                (void)hipEventCreate(&e);
                c->ev.push_back(e);
            }
        }
        e0 = c->ev[c->ev_used++];
        e1 = c->ev[c->ev_used++];
        c->timed_launches++;
    }
    unsigned long long* tin = G.coll == 2 ? c->tctr() + c->cur : nullptr;
    unsigned long long* tout = G.coll == 2 ? c->tctr() + (c->cur ^ 1) : nullptr;
    launch_lattice(c->p.storage, G, 0, c->p.variant, c->pop(c->cur), c->pop(c->cur ^ 1), c->boxes(),
                   npts > 0 ? c->toff() : nullptr, c->tlist(), c->rec(), c->partial(), (double*)c->tmax(), tin, tout,
                   s, e0, e1);
    long long off = 0;
    for (auto& st : c->sets) {
        const bool adv = st.kind == LB_COLLOIDS || st.kind == KIND_ELASTIC;
        const bool outs = st.has_model && (st.model.d_vel_out || st.model.d_vel_sum);
        if (adv || outs) {
            AdvectLaunch a;
            memset(&a, 0, sizeof(a));
            a.n = st.n;
            a.off = off;
            a.frc = st.frc;
            a.pos = (double*)st.pos;
            a.boxid = st.box;
            a.advect = adv ? 1 : 0;
            a.tin = st.kind == LB_COLLOIDS ? tin : nullptr;   // markers of curves and surfaces: no zeta'

            if (st.has_model) {
                a.vel_out = st.model.d_vel_out;
                a.vel_sum = st.model.d_vel_sum;
                a.inv_a = st.model.inv_a;
                a.inv_aL = st.model.inv_aL;
                a.mlp = st.model.d_mlp;
                for (int k = 0; k < 4; ++k) {
                    a.in_shift[k] = st.model.in_shift[k];
                    a.in_scale[k] = st.model.in_scale[k];
                }
                a.out_scale = st.model.out_scale;
            }
            launch_advect(c->p.storage, G, a, c->boxes(), c->partial(), s);
        }
        off += st.n;
    }
    c->cur ^= 1;
}

void drop_graphs(lb_ctx* c)
{
    for (auto& g : c->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    c->graphs.clear();
}

// graph of len (even) steps from the current parity; captured on first use
int get_graph(lb_ctx* c, bool rebuild, int len, hipGraphExec_t* out)
{
    for (auto& g : c->graphs)
        if (g.parity == c->cur && g.gen == c->gen && g.len == len) {
            *out = g.exec;
            return LB_OK;
        }
    if (!c->cap_stream) {
        int r = hip_check(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "hipStreamCreate");
        if (r) return r;
    }
    const int parity = c->cur;
    int r = hip_check(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
    if (r) return r;
    for (int k = 0; k < len; ++k) enqueue_step(c, c->cap_stream, rebuild);   // len even: parity restored
    hipGraph_t graph;
    r = hip_check(c, hipStreamEndCapture(c->cap_stream, &graph), "hipStreamEndCapture");
    if (r) return r;
    hipGraphExec_t exec;
    r = hip_check(c, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    if (r) {
        (void)hipGraphDestroy(graph);
        return r;
    }
    c->graphs.push_back({parity, c->gen, len, graph, exec});
    *out = exec;
    return LB_OK;
}

int check_async(lb_ctx* c)
{
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, LB_ERR_HIP, std::string("launch failed: ") + hipGetErrorString(e));
    return LB_OK;
}

}  // namespace

extern "C" {

int lb_workspace_bytes(const lb_params* p, size_t* bytes)
{
    if (!bytes) return fail(nullptr, LB_ERR_ARG, "bytes is NULL");
    Plan P;
    std::string why;
    const int r = make_plan(p, P, why);
    if (r) return fail(nullptr, r, why);
    *bytes = P.L.total;
    return LB_OK;
}

int lb_init(const lb_params* p, void* d_workspace, size_t bytes, void* hip_stream, lb_ctx** out)
{
    if (!out) return fail(nullptr, LB_ERR_ARG, "out is NULL");
    *out = nullptr;
    clear_stale_error();
    Plan P;
    std::string why;
    int r = make_plan(p, P, why);
    if (r) return fail(nullptr, r, why);
    if (!p->tau) return fail(nullptr, LB_ERR_ARG, "tau is NULL");
    for (int b = 0; b < p->nboxes; ++b)
        if (!(p->tau[b] > 0.0) || !isfinite(p->tau[b])) return fail(nullptr, LB_ERR_ARG, "tau must be finite and > 0");
    if (p->collision == LB_COLLISION_MRT && p->tau_bulk)
        for (int b = 0; b < p->nboxes; ++b)
            if (!(p->tau_bulk[b] > 0.0) || !isfinite(p->tau_bulk[b]))
                return fail(nullptr, LB_ERR_ARG, "tau_bulk must be finite and > 0");
    if (!d_workspace || ((uintptr_t)d_workspace % ALIGN) != 0)
        return fail(nullptr, LB_ERR_ARG, "workspace NULL or not 256-byte aligned");
    if (bytes < P.L.total) return fail(nullptr, LB_ERR_SIZE, "workspace too small");
    lb_ctx* c = new lb_ctx();
    c->p = *p;
    c->tau.assign(p->tau, p->tau + p->nboxes);
    c->p.tau = c->tau.data();
    c->p.tau_bulk = nullptr;   // read below, not kept
    c->P = P;
    c->ws = (char*)d_workspace;
    c->P.G.nf = c->nf();
    c->P.G.rebin = c->rebin();
    c->P.G.rebox = c->rebox();
    c->P.G.win = c->win();
    c->P.G.smax = (p->storage == LB_STORAGE_FP16 && p->nboxes == 1) ? c->smax() : nullptr;
    c->stream = (hipStream_t)hip_stream;
    c->cap_stream = nullptr;
    c->cur = 0;
    c->gen = 1;
    c->binned_gen = 0;
    c->bins_valid = false;
    c->gc_valid = false;
    c->timing = false;
    c->ev_used = 0;
    c->timed_ms = 0.0;
    c->timed_launches = 0;
    c->steps = 0;
    int e0 = p->fp16_exponent != 0 ? p->fp16_exponent : 30;
    if (p->fp16_exponent == 0 && p->kT > 0.0) {
        // thermal populations from the first step on: per population the noise of the 15 modes
        // has standard deviation at most sqrt(mu rho / w_i) <= 6 sqrt(mu rho) in units of w_i
        // (completeness of the mode basis); keep 6 of those deviations under 2^14
        const double amp = 36.0 * sqrt(3.0 * p->kT * P.G.rho0);
        e0 = std::min(30, int(floor(log2(16384.0 / amp))));
    }
    c->hboxes.resize(p->nboxes);
    for (int b = 0; b < p->nboxes; ++b) {
        BoxDev& B = c->hboxes[b];
        memset(&B, 0, sizeof(B));
        B.tau = p->tau[b];
        B.omega = 1.0 / (p->tau[b] + 0.5);
        B.tau_b = (p->collision == LB_COLLISION_MRT && p->tau_bulk) ? p->tau_bulk[b] : p->tau[b];
        B.omega_b = 1.0 / (B.tau_b + 0.5);
        // eigenvalue r of a ghost mode: the moment is multiplied by (1 - r/2) / (1 + r/2)
        const double r = p->collision == LB_COLLISION_BGK ? 1.0 / p->tau[b]
                         : p->collision == LB_COLLISION_MRT ? p->ghost_rate : 2.0;
        B.kappa_g = (1.0 - 0.5 * r) / (1.0 + 0.5 * r);
        // thermal noise: a mode whose non-equilibrium part is multiplied by gamma receives
        // variance mu rho b (1 - gamma^2), mu = kT / cs^2
        const double mu = 3.0 * p->kT;
        const double gb = 1.0 - B.omega_b, gs = 1.0 - B.omega, gg = B.kappa_g;
        B.nz_b = sqrt(mu * (1.0 - gb * gb));
        B.nz_s = sqrt(mu * (1.0 - gs * gs));
        B.nz_g = sqrt(mu * (1.0 - gg * gg));
        const double eta = P.G.rho0 * p->tau[b] / 3.0;
        B.pn = p->kT / (3.0 * M_PI * eta);
        B.inv6pe = 1.0 / (6.0 * M_PI * eta);
        B.e_data = e0;
        B.s_in = ldexpf(1.0f, -e0);
        B.s_out = ldexpf(1.0f, e0);
    }
    hipStream_t s = c->stream;
    const Geom& G = c->P.G;
    const size_t popb = (size_t)G.sbox * p->nboxes * storage_bytes(p->storage);
    launch_fill_u32(c->pop(0), (long long)(popb / 4), 0u, s);
    launch_fill_u32(c->pop(1), (long long)(popb / 4), 0u, s);
    launch_fill_u32(c->count(), G.ntiles, 0u, s);
    launch_fill_u32(c->cursor(), G.ntiles, 0u, s);
    launch_fill_u32(c->toff(), G.ntiles + 1, 0u, s);
    launch_fill_u32(c->ticket(), p->nboxes, 0u, s);
    launch_fill_u32(c->tctr(), 4, 0u, s);
    launch_fill_u32(c->tmax(), G.ntiles, 0u, s);
    launch_fill_u32(c->smax(), SMAX_SLOTS * SMAX_STRIDE, 0u, s);
    launch_fill_u32(c->errw(), 4, 0u, s);
    launch_fill_u32(c->nf(), p->nboxes, 0u, s);
    launch_fill_u32(c->rebin(), 1, 1u, s);
    launch_fill_u32(c->rebox(), p->nboxes, 1u, s);
    launch_fill_u32(c->win(), 4 * c->P.cap, 0u, s);
    r = hip_check(c, hipMemcpyAsync(c->boxes(), c->hboxes.data(), sizeof(BoxDev) * p->nboxes, hipMemcpyHostToDevice, s),
                  "hipMemcpyAsync");
    if (!r) r = check_async(c);
    if (r) {
        g_err = c->err;
        delete c;
        return r;
    }
    *out = c;
    return LB_OK;
}

int lb_set_stream(lb_ctx* c, void* hip_stream)
{
    if (!c) return LB_ERR_ARG;
    c->stream = (hipStream_t)hip_stream;
    return LB_OK;
}

int lb_set_equilibrium(lb_ctx* c, const double* d_rho, const double* d_u)
{
    if (!c) return LB_ERR_ARG;
    clear_stale_error();
    if (!d_rho || !d_u) return fail(c, LB_ERR_ARG, "lb_set_equilibrium: NULL field");
    launch_equilibrium(c->p.storage, c->P.G, c->pop(c->cur), c->boxes(), d_rho, d_u, c->stream);
    return check_async(c);
}

int lb_add_point_forces(lb_ctx* c, int64_t n, const double* d_pos, const double* d_force, const int32_t* d_box,
                        int kind, const lb_point_model* model)
{
    if (!c) return LB_ERR_ARG;
    if (n < 0) return fail(c, LB_ERR_ARG, "n < 0");
    if (n > 0 && (!d_pos || !d_force)) return fail(c, LB_ERR_ARG, "NULL positions or forces");
    if (kind != LB_FORCES_NEXT_STEP && kind != LB_FORCES_STATIC && kind != LB_COLLOIDS)
        return fail(c, LB_ERR_ARG, "unknown kind");
    if (kind == LB_COLLOIDS) {
        if (!model) return fail(c, LB_ERR_ARG, "colloids need a model (a, a_L)");
        if (!(model->inv_a > model->inv_aL) || !isfinite(model->inv_a) || !isfinite(model->inv_aL))
            return fail(c, LB_ERR_ARG, "need 1/a > 1/a_L (a < a_L) for a positive renormalised radius");
    }
    if ((int)c->sets.size() >= LB_MAX_SETS) return fail(c, LB_ERR_CAPACITY, "too many sets");
    if (total_points(c) + n > c->P.cap) return fail(c, LB_ERR_CAPACITY, "more points than max_points");
    if (n == 0) return LB_OK;
    Set s;
    s.n = n;
    s.pos = d_pos;
    s.frc = d_force;
    s.box = (const int*)d_box;
    s.kind = kind;
    s.has_model = model != nullptr;
    if (model)
        s.model = *model;
    else
        memset(&s.model, 0, sizeof(s.model));
    c->sets.push_back(s);
    c->gen++;
    c->bins_valid = false;
    c->gc_valid = false;
    return LB_OK;
}

int lb_add_elastic(lb_ctx* c, const lb_elastic* e)
{
    if (!c) return LB_ERR_ARG;
    if (!e) return fail(c, LB_ERR_ARG, "lb_add_elastic: set is NULL");
    if (e->kind != LB_ELASTIC_CHAIN && e->kind != LB_ELASTIC_SURFACE) return fail(c, LB_ERR_ARG, "unknown elastic kind");
    if (e->n <= 0 || !e->d_pos || !e->d_force) return fail(c, LB_ERR_ARG, "elastic set: n <= 0 or NULL arrays");
    if (e->kind == LB_ELASTIC_CHAIN) {
        if (e->chain_len < 2 || e->n % e->chain_len != 0)
            return fail(c, LB_ERR_ARG, "chain: chain_len >= 2 and n a multiple of it");
        if (!isfinite(e->k_spring) || !isfinite(e->l0) || e->l0 < 0.0)
            return fail(c, LB_ERR_ARG, "chain: finite k_spring and l0 >= 0");
    } else {
        if (e->ntri <= 0 || !e->d_tri || !e->d_vt_off || !e->d_vt_idx)
            return fail(c, LB_ERR_ARG, "surface: ntri > 0 and the triangle and incidence arrays");
        if (!isfinite(e->tension)) return fail(c, LB_ERR_ARG, "surface: finite tension");
        if (e->n > INT32_MAX) return fail(c, LB_ERR_ARG, "surface: too many vertices");
    }
    if ((int)c->sets.size() >= LB_MAX_SETS) return fail(c, LB_ERR_CAPACITY, "too many sets");
    if (total_points(c) + e->n > c->P.cap) return fail(c, LB_ERR_CAPACITY, "more points than max_points");
    Set s;
    s.n = e->n;
    s.pos = e->d_pos;
    s.frc = e->d_force;
    s.box = (const int*)e->d_box;
    s.kind = KIND_ELASTIC;
    memset(&s.model, 0, sizeof(s.model));
    s.model.d_vel_out = e->d_vel_out;
    s.has_model = true;   // inv_a = inv_aL = 0: the markers move with U alone
    s.el = *e;
    c->sets.push_back(s);
    c->gen++;
    c->bins_valid = false;
    c->gc_valid = false;
    return LB_OK;
}

int lb_clear_forces(lb_ctx* c)
{
    if (!c) return LB_ERR_ARG;
    c->sets.clear();
    c->gen++;
    c->bins_valid = false;
    c->gc_valid = false;
    return LB_OK;
}

int lb_step(lb_ctx* c, int32_t nsteps)
{
    if (!c) return LB_ERR_ARG;
    clear_stale_error();
    if (nsteps < 0) return fail(c, LB_ERR_ARG, "nsteps < 0");
    if (nsteps == 0) return LB_OK;
    int left = nsteps;
    force_rebin(c, c->stream);
    if (has_kind(c, LB_FORCES_NEXT_STEP)) {
        enqueue_step(c, c->stream, true);
        c->sets.erase(std::remove_if(c->sets.begin(), c->sets.end(),
                                     [](const Set& s) { return s.kind == LB_FORCES_NEXT_STEP; }),
                      c->sets.end());
        c->gen++;
        c->bins_valid = false;
        c->gc_valid = false;
        c->steps++;
        left--;
        force_rebin(c, c->stream);
    }
    const bool moving = has_kind(c, LB_COLLOIDS) || has_kind(c, KIND_ELASTIC);
    const bool pts = total_points(c) > 0;
    if (left > 0 && pts && !moving && !c->bins_valid) {
        build_points(c, c->stream);
        c->bins_valid = true;
    }
    if (left > 0 && !moving) box_update(c, c->stream, false);   // static sums outside any captured graph
    const bool rebuild = moving;
    if (c->timing || left < 4) {
        for (int k = 0; k < left; ++k) enqueue_step(c, c->stream, rebuild);
    } else {
        // the longest power-of-two chunks first
        int rest = left;
        while (rest >= 2) {
            int len = GRAPH_MAX;
            while (len > rest) len >>= 1;
            hipGraphExec_t exec;
            int r = get_graph(c, rebuild, len, &exec);
            if (r) return r;
            for (; rest >= len; rest -= len) {
                r = hip_check(c, hipGraphLaunch(exec, c->stream), "hipGraphLaunch");
                if (r) return r;
            }
        }
        if (rest) enqueue_step(c, c->stream, rebuild);
    }
    c->steps += left;
    return check_async(c);
}

int lb_prepare_steps(lb_ctx* c, int32_t nsteps)
{
    if (!c) return LB_ERR_ARG;
    clear_stale_error();
    if (nsteps < 0) return fail(c, LB_ERR_ARG, "nsteps < 0");
    // the same chunks as lb_step; a pending next-step set changes the sets after the first step
    if (has_kind(c, LB_FORCES_NEXT_STEP) || c->timing || nsteps < 4) return LB_OK;
    const bool rebuild = has_kind(c, LB_COLLOIDS) || has_kind(c, KIND_ELASTIC);
    int rest = nsteps;
    while (rest >= 2) {
        int len = GRAPH_MAX;
        while (len > rest) len >>= 1;
        hipGraphExec_t exec;
        const int r = get_graph(c, rebuild, len, &exec);
        if (r) return r;
        while (rest >= len) rest -= len;
    }
    return LB_OK;
}

static int prepare_fields(lb_ctx* c)
{
    if (total_points(c) > 0) {
        force_rebin(c, c->stream);
        elastic_forces(c, c->stream);
        build_points(c, c->stream);
        if (!has_kind(c, LB_COLLOIDS) && !has_kind(c, KIND_ELASTIC)) c->bins_valid = true;
    }
    box_update(c, c->stream, false);
    return LB_OK;
}

int lb_moments(lb_ctx* c, double* d_rho, double* d_u)
{
    if (!c) return LB_ERR_ARG;
    clear_stale_error();
    if (!d_u) return fail(c, LB_ERR_ARG, "lb_moments: d_u is NULL");
    prepare_fields(c);
    Geom G1 = c->P.G;
    G1.tpb = 1;
    launch_lattice(c->p.storage, G1, 1, 0, c->pop(c->cur), nullptr, c->boxes(),
                   total_points(c) > 0 ? c->toff() : nullptr, c->tlist(), c->rec(), d_rho, d_u, nullptr, nullptr,
                   c->stream);
    return check_async(c);
}

int lb_interp_velocity(lb_ctx* c, int64_t n, const double* d_pos, const int32_t* d_box, double* d_u_out)
{
    if (!c) return LB_ERR_ARG;
    clear_stale_error();
    if (n < 0) return fail(c, LB_ERR_ARG, "n < 0");
    if (n == 0) return LB_OK;
    if (!d_pos || !d_u_out) return fail(c, LB_ERR_ARG, "NULL positions or output");
    prepare_fields(c);
    launch_interp_points(c->p.storage, c->P.G, n, d_pos, (const int*)d_box, d_u_out, c->pop(c->cur), c->boxes(),
                         total_points(c) > 0 ? c->toff() : nullptr, c->tlist(), c->rec(), c->stream);
    return check_async(c);
}

static int read_flags(lb_ctx* c)
{
    int errw[4];
    int r = hip_check(c, hipMemcpyAsync(errw, c->errw(), sizeof(errw), hipMemcpyDeviceToHost, c->stream), "hipMemcpy");
    if (r) return r;
    std::vector<int> nf(c->p.nboxes);
    r = hip_check(c, hipMemcpyAsync(nf.data(), c->nf(), sizeof(int) * c->p.nboxes, hipMemcpyDeviceToHost, c->stream),
                  "hipMemcpy");
    if (r) return r;
    r = hip_check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (r) return r;
    if (errw[0] & 1) {
        launch_fill_u32(c->errw(), 4, 0u, c->stream);
        return fail(c, LB_ERR_ARG, "a point names a box id out of range");
    }
    if (errw[0] & 2) {
        launch_fill_u32(c->errw(), 4, 0u, c->stream);
        return fail(c, LB_ERR_NONFINITE, "non-finite point position or force");
    }
    if (errw[0] & 4) {
        launch_fill_u32(c->errw(), 4, 0u, c->stream);
        return fail(c, LB_ERR_STATE, "tile-list rebuild: a grid barrier wait ran out (lists may be incomplete)");
    }
    for (int b = 0; b < c->p.nboxes; ++b)
        if (nf[b]) return fail(c, LB_ERR_NONFINITE, "non-finite value or FP16 overflow in box " + std::to_string(b));
    return LB_OK;
}

int lb_diagnostics(lb_ctx* c, double* h_out)
{
    if (!c) return LB_ERR_ARG;
    clear_stale_error();
    if (!h_out) return fail(c, LB_ERR_ARG, "h_out is NULL");
    prepare_fields(c);
    const Geom& G = c->P.G;
    Geom G1 = G;
    G1.tpb = 1;
    launch_lattice(c->p.storage, G1, 2, 0, c->pop(c->cur), nullptr, c->boxes(), total_points(c) > 0 ? c->toff() : nullptr,
                   c->tlist(), c->rec(), c->diag(), nullptr, nullptr, nullptr, c->stream);
    launch_diag_reduce(G, c->diag(), c->diagout(), c->stream);
    int r = check_async(c);
    if (r) return r;
    r = hip_check(c,
                  hipMemcpyAsync(h_out, c->diagout(), sizeof(double) * LBD_N * c->p.nboxes, hipMemcpyDeviceToHost,
                                 c->stream),
                  "hipMemcpy");
    if (r) return r;
    r = read_flags(c);   // waits for the copy
    if (r) return r;
    for (int b = 0; b < c->p.nboxes; ++b)
        if (h_out[(size_t)b * LBD_N + 12] > 0.0)
            return fail(c, LB_ERR_NEGATIVE_DENSITY, "non-positive density in box " + std::to_string(b));
    return LB_OK;
}

int lb_sync(lb_ctx* c)
{
    if (!c) return LB_ERR_ARG;
    int r = check_async(c);
    if (r) return r;
    return read_flags(c);
}

static CkptHeader ckpt_layout(const lb_ctx* c)
{
    CkptHeader h;
    memset(&h, 0, sizeof(h));
    memcpy(h.magic, CKPT_MAGIC, 8);
    const Geom& G = c->P.G;
    h.nx = G.nx; h.ny = G.ny; h.nz = G.nz; h.nboxes = G.nboxes;
    h.storage = c->p.storage; h.collision = c->p.collision;
    h.tx = G.tx; h.ty = G.ty; h.tz = G.tz;
    h.steps = c->steps;
    h.npoints = total_points(c);
    h.pop_bytes = (int64_t)G.sbox * G.nboxes * (int64_t)storage_bytes(c->p.storage);
    h.tiles = G.ntiles;
    size_t o = align_up(sizeof(CkptHeader));
    auto take = [&](size_t b) { const size_t at = o; o = align_up(o + std::max<size_t>(b, 1)); return (int64_t)at; };
    h.off_pop = take(h.pop_bytes);
    h.off_boxes = take(sizeof(BoxDev) * G.nboxes);
    h.off_tmax = take(sizeof(float) * G.ntiles);
    h.off_smax = take(sizeof(unsigned) * SMAX_SLOTS * SMAX_STRIDE);
    h.off_tctr = take(sizeof(unsigned long long));
    h.off_nf = take(sizeof(int) * G.nboxes);
    h.off_win = take(sizeof(int4) * std::max<long long>(h.npoints, 1));
    h.total = (int64_t)o;
    return h;
}

int lb_checkpoint_bytes(const lb_ctx* c, size_t* bytes)
{
    if (!c || !bytes) return LB_ERR_ARG;
    *bytes = (size_t)ckpt_layout(c).total;
    return LB_OK;
}

int lb_checkpoint_save(lb_ctx* c, void* dst)
{
    if (!c) return LB_ERR_ARG;
    clear_stale_error();
    if (!dst || ((uintptr_t)dst % ALIGN) != 0) return fail(c, LB_ERR_ARG, "checkpoint buffer NULL or not 256-byte aligned");
    // the binning windows are part of the state once the registered sets have been binned
    if (total_points(c) > 0 && c->binned_gen != c->gen)
        return fail(c, LB_ERR_STATE, "checkpoint: step once after changing the point sets");
    c->ckpt = ckpt_layout(c);
    const CkptHeader& h = c->ckpt;
    char* d = (char*)dst;
    hipStream_t s = c->stream;
    int r = LB_OK;
    auto cp = [&](int64_t off, const void* src, size_t n) {
        if (!r) r = hip_check(c, hipMemcpyAsync(d + off, src, n, hipMemcpyDefault, s), "checkpoint copy");
    };
    cp(0, &c->ckpt, sizeof(CkptHeader));
    cp(h.off_pop, c->pop(c->cur), (size_t)h.pop_bytes);
    cp(h.off_boxes, c->boxes(), sizeof(BoxDev) * c->p.nboxes);
    cp(h.off_tmax, c->tmax(), sizeof(float) * c->P.G.ntiles);
    cp(h.off_smax, c->smax(), sizeof(unsigned) * SMAX_SLOTS * SMAX_STRIDE);
    cp(h.off_tctr, c->tctr() + c->cur, sizeof(unsigned long long));
    cp(h.off_nf, c->nf(), sizeof(int) * c->p.nboxes);
    if (h.npoints > 0) cp(h.off_win, c->win(), sizeof(int4) * h.npoints);
    return r ? r : check_async(c);
}

int lb_checkpoint_load(lb_ctx* c, const void* src)
{
    if (!c) return LB_ERR_ARG;
    clear_stale_error();
    if (!src || ((uintptr_t)src % ALIGN) != 0) return fail(c, LB_ERR_ARG, "checkpoint buffer NULL or not 256-byte aligned");
    CkptHeader h;
    int r = hip_check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (!r) r = hip_check(c, hipMemcpy(&h, src, sizeof(h), hipMemcpyDefault), "checkpoint header");
    if (r) return r;
    const CkptHeader want = ckpt_layout(c);
    if (memcmp(h.magic, CKPT_MAGIC, 8) != 0) return fail(c, LB_ERR_ARG, "not a checkpoint");
    if (h.nx != want.nx || h.ny != want.ny || h.nz != want.nz || h.nboxes != want.nboxes ||
        h.storage != want.storage || h.collision != want.collision || h.tx != want.tx || h.ty != want.ty ||
        h.tz != want.tz || h.npoints != want.npoints || h.total != want.total)
        return fail(c, LB_ERR_ARG, "checkpoint of another lattice, tiling or point count");
    const char* d = (const char*)src;
    hipStream_t s = c->stream;
    auto cp = [&](void* dst, int64_t off, size_t n) {
        if (!r) r = hip_check(c, hipMemcpyAsync(dst, d + off, n, hipMemcpyDefault, s), "checkpoint copy");
    };
    cp(c->pop(c->cur), h.off_pop, (size_t)h.pop_bytes);
    cp(c->boxes(), h.off_boxes, sizeof(BoxDev) * c->p.nboxes);
    cp(c->tmax(), h.off_tmax, sizeof(float) * c->P.G.ntiles);
    cp(c->smax(), h.off_smax, sizeof(unsigned) * SMAX_SLOTS * SMAX_STRIDE);
    cp(c->tctr() + c->cur, h.off_tctr, sizeof(unsigned long long));
    cp(c->nf(), h.off_nf, sizeof(int) * c->p.nboxes);
    if (h.npoints > 0) cp(c->win(), h.off_win, sizeof(int4) * h.npoints);
    if (r) return r;
    // rebuild the tile lists at the next step with the saved windows: the lists flag raised,
    // no box choosing new windows unless one of its points has left its window
    launch_fill_u32(c->rebin(), 1, 1u, s);
    launch_fill_u32(c->rebox(), c->p.nboxes, 0u, s);
    c->binned_gen = c->gen;
    c->bins_valid = false;
    c->gc_valid = false;
    c->steps = h.steps;
    return check_async(c);
}

int lb_destroy(lb_ctx* c)
{
    if (!c) return LB_ERR_ARG;
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    for (auto e : c->ev) (void)hipEventDestroy(e);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return LB_OK;
}

const char* lb_status_string(int status)
{
    switch (status) {
    case LB_OK: return "ok";
    case LB_ERR_ARG: return "invalid argument";
    case LB_ERR_SIZE: return "size limit or workspace too small";
    case LB_ERR_HIP: return "HIP runtime error";
    case LB_ERR_NONFINITE: return "non-finite value detected";
    case LB_ERR_CAPACITY: return "capacity exceeded";
    case LB_ERR_STATE: return "invalid state";
    case LB_ERR_NEGATIVE_DENSITY: return "non-positive density";
    }
    return "unknown status";
}

const char* lb_last_error(const lb_ctx* c) { return c ? c->err.c_str() : g_err.c_str(); }

int64_t lb_steps_taken(const lb_ctx* c) { return c ? c->steps : -1; }

int lb_kernel_timing(lb_ctx* c, int enable)
{
    if (!c) return LB_ERR_ARG;
    c->timing = enable != 0;
    c->ev_used = 0;
    c->timed_ms = 0.0;
    c->timed_launches = 0;
    return LB_OK;
}

int lb_kernel_time(lb_ctx* c, double* total_ms, int64_t* launches)
{
    if (!c || !total_ms || !launches) return LB_ERR_ARG;
    int r = hip_check(c, hipStreamSynchronize(c->stream), "hipStreamSynchronize");
    if (r) return r;
    double ms = 0.0;
    for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
        float t = 0.0f;
        r = hip_check(c, hipEventElapsedTime(&t, c->ev[k], c->ev[k + 1]), "hipEventElapsedTime");
        if (r) return r;
        ms += t;
    }
    *total_ms = ms;
    *launches = c->timed_launches;
    return LB_OK;
}

int lb_expand_multipoles(int64_t n, const int32_t* type, const double* center, const double* axis, const double* e1,
                         const double* strength, double sep, int64_t* n_out, double* pos_out, double* force_out)
{
    if (n < 0 || !n_out) return LB_ERR_ARG;
    if (n > 0 && (!type || !center || !axis || !strength || !pos_out || !force_out)) return LB_ERR_ARG;
    int64_t m = 0;
    auto put = [&](const double* R, double dr0, double dr1, double dr2, double f0, double f1, double f2) {
        pos_out[3 * m] = R[0] + dr0;
        pos_out[3 * m + 1] = R[1] + dr1;
        pos_out[3 * m + 2] = R[2] + dr2;
        force_out[3 * m] = f0;
        force_out[3 * m + 1] = f1;
        force_out[3 * m + 2] = f2;
        ++m;
    };
    const double h = 0.5 * sep;
    for (int64_t i = 0; i < n; ++i) {
        const double* R = center + 3 * i;
        const double* a = axis + 3 * i;
        const double s = strength[i];
        if (type[i] == 0) {
            put(R, 0, 0, 0, s * a[0], s * a[1], s * a[2]);
        } else if (type[i] == 1) {
            put(R, h * a[0], h * a[1], h * a[2], s * a[0], s * a[1], s * a[2]);
            put(R, -h * a[0], -h * a[1], -h * a[2], -s * a[0], -s * a[1], -s * a[2]);
        } else if (type[i] == 2) {
            if (!e1) return LB_ERR_ARG;
            const double* u = e1 + 3 * i;
            const double v[3] = {a[1] * u[2] - a[2] * u[1], a[2] * u[0] - a[0] * u[2], a[0] * u[1] - a[1] * u[0]};
            put(R, h * u[0], h * u[1], h * u[2], s * v[0], s * v[1], s * v[2]);
            put(R, -h * u[0], -h * u[1], -h * u[2], -s * v[0], -s * v[1], -s * v[2]);
            put(R, h * v[0], h * v[1], h * v[2], -s * u[0], -s * u[1], -s * u[2]);
            put(R, -h * v[0], -h * v[1], -h * v[2], s * u[0], s * u[1], s * u[2]);
        } else {
            return LB_ERR_ARG;
        }
    }
    *n_out = m;
    return LB_OK;
}

}  // extern "C"

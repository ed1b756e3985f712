// Host runtime and C ABI of the fd6 library (declared in include/fd6.h).
//
// A box borrows one caller-allocated device workspace and carves it into:
// two sets of four ghosted state fields (in / out of a substep, swapped by
// pointer as in Algorithm 2), the four RK3 register fields w, the divergence
// field of the 19-point method, reduction partials, and an FP64 staging area
// for host transfers.  In the array-of-structures layout each state set, and
// w, is one array of 4-value points instead (same bytes).  No device memory
// is allocated by the library.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <exception>
#include <type_traits>
#include <algorithm>
#include <array>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/fd6.h"
#include "fd6_internal.hpp"
#include "pack_columns.hpp"

using namespace fd6;

struct fd6_box {
    fd6_desc desc{};
    Geom geom{};
    fd6_params params{};
    bool have_params = false;
    bool have_fields = false;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    size_t tsize = 0;   // bytes per state element
    size_t wsize = 0;   // bytes per w element
    void* state[2][4] = {};
    void* w[4] = {};
    void* div = nullptr;
    double* partials = nullptr;
    double* result = nullptr;
    double* staging = nullptr;
    long long staging_elems = 0;
    int cur = 0;
    int tile = 6;  // z-sweep shape; fd6_create picks it by precision
    int zchunk = 0;  // z-sweep chunk length, 0: automatic
    // candidates timed by the last fd6_tune call: (tile, zchunk, ms per step)
    struct TuneTrial {
        int tile, zchunk;
        float ms;
    };
    std::vector<TuneTrial> tune_log;
    bool ghosts_ok[2] = {false, false};  // ghost zone of each state set is current
    std::string err;
    // optional per-launch event timing
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_kernel, ev_ghost;
    std::vector<hipEvent_t> ev_pool;
    // external force (eq. forcing): the caller's inputs, and whether the
    // device descriptor and table still have to be written
    bool force_on = false;
    bool force_dirty = false;
    fd6_forcing force{};
    void* force_dev = nullptr;
    void* force_tab = nullptr;
    // optional captured graphs of one full step, per starting parity; the
    // reducing variant also records its diagnostics target
    bool use_graph = false;
    // substeps 1 and 2 of a step in one launch (FP32, 55-point, no force)
    bool fused12 = false;
    hipStream_t cap = nullptr;  // private stream used only for graph capture
    hipGraphExec_t gstep[2] = {nullptr, nullptr};
    hipGraphExec_t gred[2] = {nullptr, nullptr};
    double* gred_out[2] = {nullptr, nullptr};
    void drop_graphs() {
        for (int i = 0; i < 2; ++i) {
            if (gstep[i]) (void)hipGraphExecDestroy(gstep[i]);
            if (gred[i]) (void)hipGraphExecDestroy(gred[i]);
            gstep[i] = gred[i] = nullptr;
            gred_out[i] = nullptr;
        }
    }
    ~fd6_box() {
        drop_graphs();
        if (cap) (void)hipStreamDestroy(cap);
        for (auto& p : ev_kernel) ev_pool.push_back(p.first), ev_pool.push_back(p.second);
        for (auto& p : ev_ghost) ev_pool.push_back(p.first), ev_pool.push_back(p.second);
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    }
};

// Ensemble of independent boxes advanced together (batched form).
struct fd6_batch {
    int n = 0;
    int precision = 0;
    int tile = 8;     // 32 x 8 z-sweep, two planes ahead
    int zchunk = 64;  // planes per work item (0: whole box)
    bool aos = false;  // every box in the array-of-structures layout
    bool use_graph = true;
    hipStream_t stream = nullptr;   // caller's stream (graph launches, transfers)
    hipStream_t cap = nullptr;      // private stream used only for graph capture
    char* ws = nullptr;
    size_t ws_bytes = 0;
    size_t tsize = 0, wsize = 0;
    std::vector<fd6_desc> desc;
    std::vector<Geom> geom;
    std::vector<fd6_params> params;
    std::vector<bool> have_fields;
    std::vector<std::array<void*, 4>> st[2], w;
    bool have_params = false;
    int parity = 0;              // state set holding the current state (all boxes)
    void* boxes_dev = nullptr;   // BatchBox<T, TW>[n]
    size_t box_bytes = 0;
    BatchItem* items_dev = nullptr;  // every workgroup's items, workgroup by workgroup
    int* wg_first_dev = nullptr;     // [grid + 1] offsets of the workgroups' lists
    long long items_cap = 0;
    int nitems = 0, grid = 0;
    double* partials = nullptr;
    double* results = nullptr;   // n x kReduceSlots
    double* staging = nullptr;
    long long staging_elems = 0;
    bool graph_ok = false;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    std::string err;
    void drop_graphs() {
        for (int i = 0; i < 2; ++i) {
            if (exec[i]) (void)hipGraphExecDestroy(exec[i]);
            if (graph[i]) (void)hipGraphDestroy(graph[i]);
            exec[i] = nullptr;
            graph[i] = nullptr;
        }
        graph_ok = false;
    }
    ~fd6_batch() {
        drop_graphs();
        if (cap) (void)hipStreamDestroy(cap);
    }
};

namespace {

constexpr size_t kAlign = 256;
// Shortest z chunk of a batch work item (each chunk re-reads 6 planes).
constexpr int kMinBatchChunk = 8;
// Schedule values of the z-chunk that select the balanced partition and the
// packed deal of whole columns.
constexpr int kBatchBalanced = -1;
constexpr int kBatchPacked = -2;

bool batch_zchunk_ok(int zchunk) {
    return zchunk == kBatchBalanced || zchunk == kBatchPacked || zchunk == 0 ||
           zchunk >= kMinBatchChunk;
}
constexpr long long kMaxFieldElems = (1LL << 31) - 1;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Plan {
    Geom g;
    size_t tsize, wsize;
    size_t off_state[2][4], off_w[4], off_div, off_partials, off_result, off_force, off_staging,
        total;
    long long staging_elems;
};

int precision_sizes(int prec, size_t* ts, size_t* wsz) {
    switch (prec) {
    case FD6_FP64: *ts = 8; *wsz = 8; return 0;
    case FD6_FP32: *ts = 4; *wsz = 4; return 0;
    case FD6_FP32_ACC64: *ts = 4; *wsz = 8; return 0;
    default: return -1;
    }
}

int validate_desc(const fd6_desc* d) {
    if (!d) return FD6_EINVAL;
    if (d->nx < 2 * kR || d->ny < 2 * kR || d->nz < 2 * kR) return FD6_EINVAL;
    if (d->nx > 4096 || d->ny > 4096 || d->nz > 4096) return FD6_EINVAL;
    if (d->flags != 0 && d->flags != FD6_LAYOUT_AOS) return FD6_EINVAL;
    if (d->variant != FD6_55P && d->variant != FD6_19P) return FD6_EINVAL;
    size_t a, b;
    if (precision_sizes(d->precision, &a, &b)) return FD6_EINVAL;
    if (d->flags == FD6_LAYOUT_AOS && d->variant != FD6_55P) return FD6_EUNSUPPORTED;
    return FD6_OK;
}

int make_plan(const fd6_desc* d, Plan* p) {
    int rc = validate_desc(d);
    if (rc) return rc;
    precision_sizes(d->precision, &p->tsize, &p->wsize);
    Geom& g = p->g;
    g.nx = d->nx;
    g.ny = d->ny;
    g.nz = d->nz;
    const long long A = 128 / (long long)p->tsize;  // elements per 128-byte line
    g.px = (int)round_up((size_t)(A + d->nx + kR), (size_t)A);
    g.plane = (long long)g.px * (d->ny + 2 * kR);
    g.origin = kR * g.plane + kR * (long long)g.px + A;
    const long long fe = g.plane * (d->nz + 2 * kR);
    g.felems = (long long)round_up((size_t)fe * p->tsize, kAlign) / (long long)p->tsize;
    const long long AW = 128 / (long long)p->wsize;
    g.wpx = (int)round_up((size_t)d->nx, (size_t)AW);
    g.wplane = (long long)g.wpx * d->ny;
    g.wfelems = (long long)round_up((size_t)(g.wplane * d->nz) * p->wsize, kAlign) /
                (long long)p->wsize;
    if (g.felems > kMaxFieldElems || g.wfelems > kMaxFieldElems) return FD6_EUNSUPPORTED;
    // array of structures: one array of 4 values per point, field q starting
    // q elements in (the same bytes as four separate fields)
    const bool aos = d->flags == FD6_LAYOUT_AOS;
    g.vs = aos ? 4 : 1;
    size_t off = 0;
    const size_t fbytes = (size_t)g.felems * p->tsize;
    const size_t wbytes = (size_t)g.wfelems * p->wsize;
    for (int s = 0; s < 2; ++s)
        for (int q = 0; q < 4; ++q)
            p->off_state[s][q] =
                aos ? off + 4 * s * fbytes + q * p->tsize : off + (4 * s + q) * fbytes;
    off += 8 * fbytes;
    for (int q = 0; q < 4; ++q) p->off_w[q] = aos ? off + q * p->wsize : off + q * wbytes;
    off += 4 * wbytes;
    p->off_div = off;
    if (d->variant == FD6_19P) off += fbytes;
    p->off_partials = off;
    off += round_up((size_t)kFusedPartials * kReduceSlots * sizeof(double), kAlign);
    p->off_result = off;
    off += kAlign;
    // force descriptor (one 256-byte block) and its per-plane table
    p->off_force = off;
    off += kAlign + round_up((size_t)2 * d->nz * sizeof(double), kAlign);
    const long long plane_c = (long long)d->nx * d->ny;
    long long st = (long long)d->nx * d->ny * d->nz;
    const long long cap = 1LL << 22;  // 32 MiB of FP64, at least one plane
    if (st > cap) st = (cap / plane_c) * plane_c;
    if (st < plane_c) st = plane_c;
    p->staging_elems = st;
    p->off_staging = off;
    off += round_up((size_t)st * sizeof(double), kAlign);
    p->total = off;
    return FD6_OK;
}

bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }
bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

template <typename H>
int hip_fail(H* b, hipError_t e, const char* what) {
    b->err = std::string(what) + ": " + hipGetErrorString(e);
    return FD6_EHIP;
}

#define HIPCHK(b, expr)                                      \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail((b), e_, #expr); \
    } while (0)

hipError_t take_event(fd6_box* b, hipEvent_t* e) {
    if (!b->ev_pool.empty()) {
        *e = b->ev_pool.back();
        b->ev_pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

// Records an event pair around the launches made by f when timing is on.
template <typename F>
int timed(fd6_box* b, std::vector<std::pair<hipEvent_t, hipEvent_t>>& log, F&& f) {
    if (!b->timing) return f();
    hipEvent_t e0, e1;
    HIPCHK(b, take_event(b, &e0));
    HIPCHK(b, take_event(b, &e1));
    HIPCHK(b, hipEventRecord(e0, b->stream));
    int rc = f();
    HIPCHK(b, hipEventRecord(e1, b->stream));
    log.emplace_back(e0, e1);
    return rc;
}

// RK3 coefficients of the 2N-storage scheme (Williamson 1980), alpha(1) = 0.
constexpr double kAlpha[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
constexpr double kBeta[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};

template <typename T>
Coef<T> make_coef(const fd6_params& p) {
    const double h[3] = {p.dx, p.dy, p.dz};
    const double w1[3] = {45.0, -9.0, 1.0};
    const double w2[4] = {-490.0, 270.0, -27.0, 2.0};
    const double wm[3] = {270.0, -27.0, 2.0};
    Coef<T> c{};
    double d2[3][4];
    for (int a = 0; a < 3; ++a) {
        for (int k = 0; k < 3; ++k) c.d1[a][k] = T(w1[k] / (60.0 * h[a]));
        for (int k = 0; k < 4; ++k) {
            d2[a][k] = w2[k] / (180.0 * h[a] * h[a]);
            c.d2[a][k] = T(d2[a][k]);
            c.lp[a][k] = T(p.nu * d2[a][k]);
        }
    }
    const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};  // xy, xz, yz
    for (int q = 0; q < 3; ++q)
        for (int k = 0; k < 3; ++k) {
            const double m = wm[k] / (720.0 * h[pa[q]] * h[pb[q]]);
            c.mx[q][k] = T(m);
            c.mw[q][k] = T(p.nu * m / 3.0);
        }
    for (int i = 0; i < 3; ++i)
        for (int a = 0; a < 3; ++a)
            for (int k = 0; k < 4; ++k)
                c.lw[i][a][k] = T(p.nu * (a == i ? 4.0 / 3.0 : 1.0) * d2[a][k]);
    c.nu = T(p.nu);
    c.cs2 = T(p.cs * p.cs);
    c.nu3 = p.nu / 3.0;
    double sg[3], sg4[3];
    for (int a = 0; a < 3; ++a) {
        sg[a] = p.nu / (180.0 * h[a] * h[a]);
        sg4[a] = (4.0 / 3.0) * sg[a];
        c.sg[a] = T(sg[a]);
        c.sg4[a] = T(sg4[a]);
    }
    for (int i = 0; i < 3; ++i) {
        const double sx = i == 0 ? sg4[0] : sg[0], sy = i == 1 ? sg4[1] : sg[1];
        c.kxy[i] = T(-490.0 * (sx + sy));
    }
    for (int q = 0; q < 3; ++q) c.mu[q] = T(p.nu / (3.0 * 720.0 * h[pa[q]] * h[pb[q]]));
    c.kp = T(-490.0 * (sg[0] + sg[1]));
    return c;
}

template <typename T>
Fields4<T> fields_of(void* const f[4]) {
    Fields4<T> r;
    for (int q = 0; q < 4; ++q) r.f[q] = static_cast<T*>(f[q]);
    return r;
}

// One substep: boundary condition (the ghost pass runs only for kernels that
// read the ghost zone and only when it is stale), the substep kernel(s), and
// the in/out swap.  With red_out != nullptr (substep 3) the FP64 diagnostics
// of the new state are written to red_out (device, 5 doubles).
template <typename T, typename TW>
int do_substep(fd6_box* b, int s, const RKCoef<TW>& rk, double* red_out = nullptr) {
    const Geom& g = b->geom;
    Fields4<T> in = fields_of<T>(b->state[b->cur]);
    Fields4<T> out = fields_of<T>(b->state[b->cur ^ 1]);
    Fields4<TW> w = fields_of<TW>(b->w);
    const Coef<T> c = make_coef<T>(b->params);
    const bool needs_ghosts = substep55_reads_ghosts(b->tile);
    int rc = FD6_OK;
    if (needs_ghosts && !b->ghosts_ok[b->cur]) {
        rc = timed(b, b->ev_ghost, [&]() -> int {
            HIPCHK(b, launch_ghost_fill<T>(g, in, 4, b->stream));
            return FD6_OK;
        });
        if (rc) return rc;
        b->ghosts_ok[b->cur] = true;
    }
    int nparts = 0;  // > 0: substep 3 wrote the diagnostics partials itself
    const ForceArgs<T> fa{static_cast<const ForceDev<T>*>(b->force_dev),
                          static_cast<const T*>(b->force_tab)};
    const ForceArgs<T>* frc = b->force_on ? &fa : nullptr;
    if (b->desc.variant == FD6_55P) {
        double* parts = (red_out && s == 3) ? b->partials : nullptr;
        auto launch = g.vs == 4 ? launch_substep55_aos<T, TW> : launch_substep55<T, TW>;
        rc = timed(b, b->ev_kernel, [&]() -> int {
            HIPCHK(b, launch(g, in, out, w, c, rk, s, b->tile, b->zchunk, parts, kFusedPartials,
                             &nparts, frc, b->stream));
            return FD6_OK;
        });
        if (rc) return rc;
    } else {
        T* dv = static_cast<T*>(b->div);
        rc = timed(b, b->ev_kernel, [&]() -> int {
            HIPCHK(b, (launch_pass19a<T, TW>(g, in, out, w, dv, c, rk, s, b->tile, b->zchunk,
                                             frc, b->stream)));
            return FD6_OK;
        });
        if (rc) return rc;
        if (needs_ghosts) {  // the direct pass 2 reads the divergence's ghost zone
            Fields4<T> d1{{dv, dv, dv, dv}};
            rc = timed(b, b->ev_ghost, [&]() -> int {
                HIPCHK(b, launch_ghost_fill<T>(g, d1, 1, b->stream));
                return FD6_OK;
            });
            if (rc) return rc;
        }
        double* parts = (red_out && s == 3) ? b->partials : nullptr;
        rc = timed(b, b->ev_kernel, [&]() -> int {
            HIPCHK(b, (launch_pass19b<T, TW>(g, dv, out, w, c, rk, s, b->tile, b->zchunk, parts,
                                             kFusedPartials, &nparts, b->stream)));
            return FD6_OK;
        });
        if (rc) return rc;
    }
    b->ghosts_ok[b->cur ^ 1] = false;  // no kernel writes the output ghost zone
    b->cur ^= 1;
    if (red_out && s == 3) {
        const double dV = b->params.dx * b->params.dy * b->params.dz;
        if (nparts > 0)
            HIPCHK(b, launch_reduce_final(b->partials, nparts, red_out, dV, b->stream));
        else
            HIPCHK(b, launch_reduce<T>(g, fields_of<T>(b->state[b->cur]), b->partials, red_out,
                                       dV, b->stream));
    }
    return FD6_OK;
}

// Writes the force descriptor and table for the current parameters if the
// force or the parameters changed since the last write (stream-ordered, and
// never inside a captured step, so replays read the current force).
template <typename T>
int force_sync(fd6_box* b) {
    if (!b->force_on || !b->force_dirty) return FD6_OK;
    const fd6_forcing& f = b->force;
    const fd6_params& pp = b->params;
    const double k[3] = {f.kx, f.ky, f.kz}, e[3] = {f.ex, f.ey, f.ez};
    const double kk = std::sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    const double ke = k[0] * e[0] + k[1] * e[1] + k[2] * e[2];
    // eq. (forcing): N = f0 cs sqrt(|k| cs / dt), f_k = (k x e) / sqrt(|k|^2 - (k.e)^2)
    const double norm = f.f0 * pp.cs * std::sqrt(kk * pp.cs / pp.dt);
    const double den = std::sqrt(kk * kk - ke * ke);
    const double kxe[3] = {k[1] * e[2] - k[2] * e[1], k[2] * e[0] - k[0] * e[2],
                           k[0] * e[1] - k[1] * e[0]};
    const double a[3] = {norm * kxe[0] / den, norm * kxe[1] / den, norm * kxe[2] / den};
    const double h[3] = {pp.dx, pp.dy, pp.dz};
    HIPCHK(b, launch_force_table<T>(b->geom, static_cast<ForceDev<T>*>(b->force_dev),
                                    static_cast<T*>(b->force_tab), k, f.phase, h, a, b->stream));
    b->force_dirty = false;
    return FD6_OK;
}

// Whether a step runs substeps 1 and 2 as one fused launch (fd6_set_fused_substeps).
bool fused_step(const fd6_box* b) { return b->fused12 && !b->force_on; }

// Substeps 1 and 2 in one launch: state[cur] -> state[cur ^ 1], w holding
// the substep-2 register (one in/out swap instead of two).
template <typename T, typename TW>
int fused12_substeps(fd6_box* b) {
    if constexpr (!std::is_same<T, float>::value || !std::is_same<TW, float>::value) {
        b->err = "fused substeps: FP32 state and register only";
        return FD6_EUNSUPPORTED;
    } else {
        const double dt = b->params.dt;
        const RKCoef<TW> rk1{TW(kAlpha[0]), TW(kBeta[0]), TW(dt)};
        const RKCoef<TW> rk2{TW(kAlpha[1]), TW(kBeta[1]), TW(dt)};
        const Coef<T> c = make_coef<T>(b->params);
        int rc = timed(b, b->ev_kernel, [&]() -> int {
            HIPCHK(b, (launch_fused12<T, TW>(b->geom, fields_of<T>(b->state[b->cur]),
                                             fields_of<T>(b->state[b->cur ^ 1]),
                                             fields_of<TW>(b->w), c, rk1, rk2, b->zchunk,
                                             b->stream)));
            return FD6_OK;
        });
        if (rc) return rc;
        b->ghosts_ok[b->cur ^ 1] = false;
        b->cur ^= 1;
        return FD6_OK;
    }
}

// One full step (Algorithm 2: three substeps); red_out != nullptr also
// produces the diagnostics of the new state.
template <typename T, typename TW>
int one_step(fd6_box* b, double* red_out) {
    const double dt = b->params.dt;
    int s0 = 0;
    if (fused_step(b)) {
        int rc = fused12_substeps<T, TW>(b);
        if (rc) return rc;
        s0 = 2;
    }
    for (int s = s0; s < 3; ++s) {
        RKCoef<TW> rk{TW(kAlpha[s]), TW(kBeta[s]), TW(dt)};
        int rc = do_substep<T, TW>(b, s + 1, rk, red_out);
        if (rc) return rc;
    }
    return FD6_OK;
}

// Captures one full step starting from state set `parity` into *out.  The
// capture runs on a private stream; a kernel shape that reads ghost zones
// records a ghost pass in every substep (the lazy bookkeeping cannot follow
// replays).  The box's stream, parity and ghost flags are restored.
template <typename T, typename TW>
int capture_step(fd6_box* b, int parity, double* red_out, hipGraphExec_t* out) {
    if (!b->cap) HIPCHK(b, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    hipStream_t user = b->stream;
    const int cur = b->cur;
    b->stream = b->cap;
    b->cur = parity;
    b->ghosts_ok[0] = b->ghosts_ok[1] = false;
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    int rc = e == hipSuccess ? one_step<T, TW>(b, red_out) : FD6_OK;
    hipGraph_t g = nullptr;
    hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(b->cap, &g) : e;
    b->stream = user;
    b->cur = cur;
    b->ghosts_ok[0] = b->ghosts_ok[1] = false;
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e2 != hipSuccess) return hip_fail(b, e2, "graph capture of one step");
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(b, e, "hipGraphInstantiate");
    return FD6_OK;
}

template <typename T, typename TW>
int do_steps(fd6_box* b, int nsteps, double* red_out = nullptr) {
    int frc = force_sync<T>(b);
    if (frc) return frc;
    if (!b->use_graph || b->timing) {
        for (int n = 0; n < nsteps; ++n) {
            int rc = one_step<T, TW>(b, n == nsteps - 1 ? red_out : nullptr);
            if (rc) return rc;
        }
        return FD6_OK;
    }
    for (int n = 0; n < nsteps; ++n) {
        const bool red = red_out && n == nsteps - 1;
        const int p = b->cur;
        hipGraphExec_t* x = red ? &b->gred[p] : &b->gstep[p];
        if (red && *x && b->gred_out[p] != red_out) {
            (void)hipGraphExecDestroy(*x);
            *x = nullptr;
        }
        if (!*x) {
            int rc = capture_step<T, TW>(b, p, red ? red_out : nullptr, x);
            if (rc) return rc;
            if (red) b->gred_out[p] = red_out;
        }
        HIPCHK(b, hipGraphLaunch(*x, b->stream));
        if (!fused_step(b)) b->cur ^= 1;  // three in/out swaps (two when fused)
        b->ghosts_ok[0] = b->ghosts_ok[1] = false;
    }
    return FD6_OK;
}

template <typename T, typename TW>
int do_rhs(fd6_box* b, double* const out[4]) {
    // substep-1 arithmetic with dt = 1 leaves w = r; the result state is
    // discarded by not swapping back
    RKCoef<TW> rk{TW(0), TW(0), TW(1)};
    int rc = force_sync<T>(b);
    if (rc) return rc;
    rc = do_substep<T, TW>(b, 1, rk);
    if (rc) return rc;  // a failed substep returns before its in/out swap
    b->cur ^= 1;        // keep the original state current
    b->ghosts_ok[b->cur ^ 1] = false;
    const Geom& g = b->geom;
    // export in z-chunks of whole planes that fit the staging area
    const long long plane_c = (long long)g.nx * g.ny;
    const int chunk = (int)(b->staging_elems / plane_c);
    for (int q = 0; q < 4; ++q) {
        const TW* src = static_cast<const TW*>(b->w[q]);
        for (int z = 0; z < g.nz; z += chunk) {
            const int np = (z + chunk <= g.nz) ? chunk : g.nz - z;
            HIPCHK(b, launch_export_w<TW>(g, src, b->staging, z, np, b->stream));
            HIPCHK(b, hipMemcpyAsync(out[q] + (long long)z * plane_c, b->staging,
                                     (size_t)np * plane_c * sizeof(double),
                                     hipMemcpyDeviceToHost, b->stream));
            HIPCHK(b, hipStreamSynchronize(b->stream));
        }
    }
    return FD6_OK;
}

template <typename T>
int import_host(fd6_box* b, const double* const src[4]) {
    const Geom& g = b->geom;
    const long long plane_c = (long long)g.nx * g.ny;
    const int chunk = (int)(b->staging_elems / plane_c);
    for (int q = 0; q < 4; ++q) {
        T* dst = static_cast<T*>(b->state[b->cur][q]);
        for (int z = 0; z < g.nz; z += chunk) {
            const int np = (z + chunk <= g.nz) ? chunk : g.nz - z;
            HIPCHK(b, hipMemcpyAsync(b->staging, src[q] + (long long)z * plane_c,
                                     (size_t)np * plane_c * sizeof(double), hipMemcpyHostToDevice,
                                     b->stream));
            HIPCHK(b, launch_import<T>(g, b->staging, dst, z, np, b->stream));
            HIPCHK(b, hipStreamSynchronize(b->stream));
        }
    }
    return FD6_OK;
}

template <typename T>
int export_host(fd6_box* b, double* const dst[4]) {
    const Geom& g = b->geom;
    const long long plane_c = (long long)g.nx * g.ny;
    const int chunk = (int)(b->staging_elems / plane_c);
    for (int q = 0; q < 4; ++q) {
        const T* src = static_cast<const T*>(b->state[b->cur][q]);
        for (int z = 0; z < g.nz; z += chunk) {
            const int np = (z + chunk <= g.nz) ? chunk : g.nz - z;
            HIPCHK(b, launch_export<T>(g, src, b->staging, z, np, b->stream));
            HIPCHK(b, hipMemcpyAsync(dst[q] + (long long)z * plane_c, b->staging,
                                     (size_t)np * plane_c * sizeof(double), hipMemcpyDeviceToHost,
                                     b->stream));
            HIPCHK(b, hipStreamSynchronize(b->stream));
        }
    }
    return FD6_OK;
}

template <typename T>
int import_device(fd6_box* b, const double* const src[4]) {
    for (int q = 0; q < 4; ++q)
        HIPCHK(b, launch_import<T>(b->geom, src[q], static_cast<T*>(b->state[b->cur][q]), 0,
                                   b->geom.nz, b->stream));
    return FD6_OK;
}

template <typename T>
int export_device(fd6_box* b, double* const dst[4]) {
    for (int q = 0; q < 4; ++q)
        HIPCHK(b, launch_export<T>(b->geom, static_cast<const T*>(b->state[b->cur][q]), dst[q], 0,
                                   b->geom.nz, b->stream));
    return FD6_OK;
}

int reset_w(fd6_box* b) {
    if (b->wsize == 8)
        HIPCHK(b, launch_zero_w<double>(b->geom, fields_of<double>(b->w), b->stream));
    else
        HIPCHK(b, launch_zero_w<float>(b->geom, fields_of<float>(b->w), b->stream));
    return FD6_OK;
}

template <typename T>
int do_reduce(fd6_box* b, fd6_reductions* out) {
    const Geom& g = b->geom;
    const double dV = b->params.dx * b->params.dy * b->params.dz;
    HIPCHK(b, launch_reduce<T>(g, fields_of<T>(b->state[b->cur]), b->partials, b->result, dV,
                               b->stream));
    double r[kReduceSlots];
    HIPCHK(b, hipMemcpyAsync(r, b->result, 5 * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    out->mass = r[0];
    out->kinetic_energy = r[1];
    out->sum_lnrho = r[2];
    out->umax = r[3];
    out->nonfinite = (int64_t)r[4];
    return out->nonfinite > 0 ? FD6_ENONFINITE : FD6_OK;
}

template <typename T>
int do_reduce_device(fd6_box* b, double* d_out) {
    const Geom& g = b->geom;
    const double dV = b->params.dx * b->params.dy * b->params.dz;
    HIPCHK(b, launch_reduce<T>(g, fields_of<T>(b->state[b->cur]), b->partials, d_out, dV,
                               b->stream));
    return FD6_OK;
}

// Precision dispatch: FP64 -> (double, double); FP32 -> (float, float);
// FP32 state with FP64 RK3 register -> (float, double).
template <typename F>
int dispatch(fd6_box* b, F&& f) {
    switch (b->desc.precision) {
    case FD6_FP64: return f((double*)nullptr, (double*)nullptr);
    case FD6_FP32: return f((float*)nullptr, (float*)nullptr);
    default: return f((float*)nullptr, (double*)nullptr);
    }
}

template <typename H, typename F>
int guarded(H* b, F&& f) {
    try {
        return f();
    } catch (const std::bad_alloc&) {
        if (b) b->err = "host allocation failed";
        return FD6_ENOMEM;
    } catch (const std::exception& e) {
        if (b) b->err = e.what();
        return FD6_EHIP;
    } catch (...) {
        if (b) b->err = "unknown exception";
        return FD6_EHIP;
    }
}

bool ready(fd6_box* b) { return b->have_params && b->have_fields; }


// ---------------------------------------------------------------------------
// Batched ensemble
// ---------------------------------------------------------------------------

struct BatchPlan {
    std::vector<Plan> box;
    std::vector<size_t> base;  // workspace offset of each box's fields
    size_t off_boxes, off_items, off_wg, off_partials, off_results, off_staging, total;
    size_t box_bytes;
    long long items_cap, staging_elems;
};

size_t batch_box_bytes(int prec) {
    switch (prec) {
    case FD6_FP64: return sizeof(BatchBox<double, double>);
    case FD6_FP32: return sizeof(BatchBox<float, float>);
    default: return sizeof(BatchBox<float, double>);
    }
}

int make_batch_plan(int n, const fd6_desc* d, BatchPlan* bp) {
    if (n < 1 || n > 65536 || !d) return FD6_EINVAL;
    bp->box.resize(n);
    bp->base.resize(n);
    size_t off = 0;
    long long items = 0, stag = 0;
    for (int i = 0; i < n; ++i) {
        int rc = make_plan(&d[i], &bp->box[i]);
        if (rc) return rc;
        if (d[i].precision != d[0].precision) return FD6_EINVAL;
        if (d[i].variant != FD6_55P) return FD6_EUNSUPPORTED;
        if (d[i].flags != d[0].flags) return FD6_EINVAL;  // one layout per ensemble
        bp->base[i] = off;
        // this box's state and w fields (the per-box plan puts them first)
        off += bp->box[i].off_div;
        // work items of the smallest tile extents (x 32, y 4) with chunks of at
        // least kMinBatchChunk planes (an even split into ceil(nz / zchunk)
        // chunks never makes more than ceil(nz / kMinBatchChunk))
        items += (long long)((d[i].nx + 31) / 32) * ((d[i].ny + 3) / 4) *
                 ((d[i].nz + kMinBatchChunk - 1) / kMinBatchChunk);
        const long long pc = (long long)d[i].nx * d[i].ny;
        long long st = std::min<long long>(pc * d[i].nz, std::max<long long>(pc, 1LL << 22));
        stag = std::max(stag, st);
    }
    bp->box_bytes = batch_box_bytes(d[0].precision);
    bp->off_boxes = off;
    off += round_up(bp->box_bytes * n, kAlign);
    // a balanced partition adds at most one split per workgroup
    items += kMaxBatchGrid;
    bp->items_cap = items;
    bp->off_items = off;
    off += round_up(sizeof(BatchItem) * items, kAlign);
    bp->off_wg = off;
    off += round_up(sizeof(int) * (kMaxBatchGrid + 1), kAlign);
    bp->off_partials = off;
    off += round_up((size_t)kReduceBlocks * kReduceSlots * sizeof(double), kAlign);
    bp->off_results = off;
    off += round_up((size_t)n * kReduceSlots * sizeof(double), kAlign);
    bp->staging_elems = stag;
    bp->off_staging = off;
    off += round_up((size_t)stag * sizeof(double), kAlign);
    bp->total = off;
    return FD6_OK;
}

// Per-box descriptors (geometry, both state sets, w, coefficients, dt).
template <typename T, typename TW>
int upload_boxes(fd6_batch* b) {
    std::vector<BatchBox<T, TW>> h(b->n);
    for (int i = 0; i < b->n; ++i) {
        h[i].g = b->geom[i];
        h[i].st[0] = fields_of<T>(b->st[0][i].data());
        h[i].st[1] = fields_of<T>(b->st[1][i].data());
        h[i].w = fields_of<TW>(b->w[i].data());
        h[i].cf = make_coef<T>(b->params[i]);
        h[i].dt = TW(b->params[i].dt);
    }
    HIPCHK(b, hipMemcpyAsync(b->boxes_dev, h.data(), sizeof(BatchBox<T, TW>) * b->n,
                             hipMemcpyHostToDevice, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    return FD6_OK;
}

// Work lists for kernel shape `tile` and chunk length `zchunk`, one list per
// workgroup of the persistent grid (workgroup L = remapped block index, so a
// range of L lies on one XCD).
//  * zchunk >= 0: every box's z range split evenly into chunks of at most
//    zchunk planes (0: whole columns); all tile-chunks sorted longest first
//    (then box, z, y, x), and workgroup L takes entries L, L + G, L + 2G, ...
//    The first G entries are neighbouring tiles, swept at the same time.
//  * zchunk = kBatchBalanced: the tile columns of all boxes in order (box, y,
//    x), cut into G runs of equal cost (planes swept, 6 more per column piece
//    for the pipeline refill); workgroup L sweeps run L, so every workgroup
//    has the same work, and a column is split only where a run ends (pieces
//    of at least kMinBatchChunk planes).
//  * zchunk = kBatchPacked: whole tile columns, longest first, each dealt to
//    the least-loaded workgroup (pack_columns); only a column that would take
//    its workgroup past a target cost is split.
// The batch's schedule, lists and grid change only when the lists are built
// and uploaded; a refused schedule leaves the previous one in force.
template <typename T, typename TW>
int build_items(fd6_batch* b, int tile, int zchunk) {
    int tx = 0, ty = 0;
    if (substep55_tile_dims(tile, &tx, &ty)) return FD6_EINVAL;
    if (!batch_zchunk_ok(zchunk)) return FD6_EINVAL;
    // persistent grid: every resident workgroup, a multiple of the 8 XCDs
    int dev = 0, cus = 0;
    HIPCHK(b, hipGetDevice(&dev));
    HIPCHK(b, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int per_cu = b->aos ? batch55_blocks_per_cu_aos<T, TW>(tile)
                              : batch55_blocks_per_cu<T, TW>(tile);
    long long resident = std::min<long long>((long long)cus * per_cu, kMaxBatchGrid);
    const long long pieces = 8;  // keep G a multiple of the XCD count
    std::vector<BatchItem> flat;
    std::vector<int> first;
    if (zchunk == kBatchPacked) {
        std::vector<BatchItem> cols;
        for (int i = 0; i < b->n; ++i) {
            const Geom& g = b->geom[i];
            for (int y0 = 0; y0 < g.ny; y0 += ty)
                for (int x0 = 0; x0 < g.nx; x0 += tx)
                    cols.push_back(BatchItem{i, x0, y0, 0, g.nz});
        }
        const long long gsz = resident >= pieces ? resident / pieces * pieces : resident;
        pack_columns(cols, (int)std::max<long long>(gsz, 1), 2 * kR, kMinBatchChunk, &flat,
                     &first);
        if ((long long)flat.size() > b->items_cap) {
            b->err = "work list larger than the workspace's item capacity";
            return FD6_EUNSUPPORTED;
        }
    } else if (zchunk != kBatchBalanced) {
        std::vector<BatchItem> it;
        std::vector<long long> cost;
        for (int i = 0; i < b->n; ++i) {
            const Geom& g = b->geom[i];
            // chunks of at most zchunk planes, split evenly (96 planes with
            // 64-plane chunks give 48 + 48, not 64 + 32)
            const int cap = zchunk > 0 ? std::min(zchunk, g.nz) : g.nz;
            const int nch = (g.nz + cap - 1) / cap;
            const int zl = (g.nz + nch - 1) / nch;
            for (int zb = 0; zb < g.nz; zb += zl)
                for (int y0 = 0; y0 < g.ny; y0 += ty)
                    for (int x0 = 0; x0 < g.nx; x0 += tx) {
                        it.push_back(BatchItem{i, x0, y0, zb, std::min(zb + zl, g.nz)});
                        cost.push_back((long long)(std::min(zb + zl, g.nz) - zb + 2 * kR));
                    }
        }
        // the workspace holds the lists of the smallest tile with chunks of
        // kMinBatchChunk planes, so this cannot trigger for an accepted schedule
        if ((long long)it.size() > b->items_cap) {
            b->err = "work list larger than the workspace's item capacity";
            return FD6_EUNSUPPORTED;
        }
        std::vector<int> order(it.size());
        for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int c) { return cost[a] > cost[c]; });
        long long gsz = std::min<long long>(resident, (long long)it.size());
        if (gsz >= pieces) gsz = gsz / pieces * pieces;
        const int G = (int)std::max<long long>(gsz, 1);
        flat.reserve(it.size());
        first.assign(G + 1, 0);
        for (int L = 0; L < G; ++L) {
            first[L] = (int)flat.size();
            for (size_t k = L; k < order.size(); k += G) flat.push_back(it[order[k]]);
        }
        first[G] = (int)flat.size();
    } else {
        struct Col {
            int box, x0, y0, nz;
        };
        std::vector<Col> cols;
        long long total = 0;
        for (int i = 0; i < b->n; ++i) {
            const Geom& g = b->geom[i];
            for (int y0 = 0; y0 < g.ny; y0 += ty)
                for (int x0 = 0; x0 < g.nx; x0 += tx) {
                    cols.push_back(Col{i, x0, y0, g.nz});
                    total += g.nz + 2 * kR;
                }
        }
        long long gsz = resident >= pieces ? resident / pieces * pieces : resident;
        const int G = (int)std::max<long long>(gsz, 1);
        first.assign(G + 1, 0);
        // Each run aims at the mean of the cost still unassigned over the
        // runs still open (counting one refill per column not yet started and
        // one per split still to come), so no shortfall piles up at the end.
        long long left = total;  // planes + one refill per column, unassigned
        int L = 0;
        long long load = 0;
        auto mean_left = [&]() { return (double)(left + (long long)(G - L - 1) * 2 * kR) / (G - L); };
        double target = mean_left();
        for (const Col& c : cols) {
            int z = 0;
            bool first_piece = true;
            while (z < c.nz) {
                const int rem = c.nz - z;
                const double room = target - (double)load - 2 * kR;  // planes that fit
                int take = rem;
                if (L < G - 1 && rem > room) {
                    take = (int)std::lround(room);
                    if (take < kMinBatchChunk) {
                        if (load > 0) {  // close this run; the piece opens the next
                            first[++L] = (int)flat.size();
                            load = 0;
                            target = mean_left();
                            continue;
                        }
                        take = std::min(rem, kMinBatchChunk);
                    } else if (rem - take < kMinBatchChunk) {
                        // a split here would leave too short a piece: split
                        // earlier (short of the target) or take it all (past it)
                        const double under = room - (rem - kMinBatchChunk), over = rem - room;
                        take = (rem - kMinBatchChunk >= kMinBatchChunk && under < over)
                                   ? rem - kMinBatchChunk
                                   : rem;
                    }
                }
                flat.push_back(BatchItem{c.box, c.x0, c.y0, z, z + take});
                load += take + 2 * kR;
                left -= take + (first_piece ? 2 * kR : 0);
                first_piece = false;
                z += take;
                if (L < G - 1 && (double)load >= target - 0.5) {
                    first[++L] = (int)flat.size();
                    load = 0;
                    target = mean_left();
                }
            }
        }
        for (int k = L + 1; k <= G; ++k) first[k] = (int)flat.size();
        if ((long long)flat.size() > b->items_cap) {
            b->err = "work list larger than the workspace's item capacity";
            return FD6_EUNSUPPORTED;
        }
    }
    HIPCHK(b, hipMemcpyAsync(b->items_dev, flat.data(), sizeof(BatchItem) * flat.size(),
                             hipMemcpyHostToDevice, b->stream));
    HIPCHK(b, hipMemcpyAsync(b->wg_first_dev, first.data(), sizeof(int) * first.size(),
                             hipMemcpyHostToDevice, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    b->tile = tile;
    b->zchunk = zchunk;
    b->nitems = (int)flat.size();
    b->grid = (int)first.size() - 1;
    b->drop_graphs();
    return FD6_OK;
}

template <typename T, typename TW>
int batch_substeps(fd6_batch* b, hipStream_t st, int parity) {
    auto launch = b->aos ? launch_batch55_aos<T, TW> : launch_batch55<T, TW>;
    for (int s = 0; s < 3; ++s) {
        HIPCHK(b, launch(static_cast<const BatchBox<T, TW>*>(b->boxes_dev), b->items_dev,
                         b->wg_first_dev, b->grid, parity, s + 1, b->tile, TW(kAlpha[s]),
                         TW(kBeta[s]), st));
        parity ^= 1;
    }
    return FD6_OK;
}

// One graph per starting parity: substeps 1-3 of a full step.
template <typename T, typename TW>
int build_graphs(fd6_batch* b) {
    b->drop_graphs();
    if (!b->cap) HIPCHK(b, hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    for (int p = 0; p < 2; ++p) {
        HIPCHK(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
        int rc = batch_substeps<T, TW>(b, b->cap, p);
        hipGraph_t gr = nullptr;
        hipError_t e = hipStreamEndCapture(b->cap, &gr);
        if (rc) {
            if (gr) (void)hipGraphDestroy(gr);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(b, e, "hipStreamEndCapture");
        b->graph[p] = gr;
        HIPCHK(b, hipGraphInstantiate(&b->exec[p], gr, nullptr, nullptr, 0));
    }
    b->graph_ok = true;
    return FD6_OK;
}

template <typename T, typename TW>
int batch_steps(fd6_batch* b, int nsteps) {
    if (b->nitems == 0) {
        int rc = build_items<T, TW>(b, b->tile, b->zchunk);
        if (rc) return rc;
    }
    if (b->use_graph && !b->graph_ok) {
        int rc = build_graphs<T, TW>(b);
        if (rc) return rc;
    }
    for (int n = 0; n < nsteps; ++n) {
        if (b->use_graph) {
            HIPCHK(b, hipGraphLaunch(b->exec[b->parity], b->stream));
        } else {
            int rc = batch_substeps<T, TW>(b, b->stream, b->parity);
            if (rc) return rc;
        }
        b->parity ^= 1;
    }
    return FD6_OK;
}

template <typename F>
int batch_dispatch(fd6_batch* b, F&& f) {
    switch (b->precision) {
    case FD6_FP64: return f((double*)nullptr, (double*)nullptr);
    case FD6_FP32: return f((float*)nullptr, (float*)nullptr);
    default: return f((float*)nullptr, (double*)nullptr);
    }
}

template <typename T>
int batch_import(fd6_batch* b, int i, const double* const src[4]) {
    const Geom& g = b->geom[i];
    const long long plane_c = (long long)g.nx * g.ny;
    const int chunk = (int)std::max<long long>(1, b->staging_elems / plane_c);
    for (int q = 0; q < 4; ++q) {
        T* dst = static_cast<T*>(b->st[b->parity][i][q]);
        for (int z = 0; z < g.nz; z += chunk) {
            const int np = (z + chunk <= g.nz) ? chunk : g.nz - z;
            HIPCHK(b, hipMemcpyAsync(b->staging, src[q] + (long long)z * plane_c,
                                     (size_t)np * plane_c * sizeof(double), hipMemcpyHostToDevice,
                                     b->stream));
            HIPCHK(b, launch_import<T>(g, b->staging, dst, z, np, b->stream));
            HIPCHK(b, hipStreamSynchronize(b->stream));
        }
    }
    return FD6_OK;
}

template <typename T>
int batch_export(fd6_batch* b, int i, double* const dst[4]) {
    const Geom& g = b->geom[i];
    const long long plane_c = (long long)g.nx * g.ny;
    const int chunk = (int)std::max<long long>(1, b->staging_elems / plane_c);
    for (int q = 0; q < 4; ++q) {
        const T* src = static_cast<const T*>(b->st[b->parity][i][q]);
        for (int z = 0; z < g.nz; z += chunk) {
            const int np = (z + chunk <= g.nz) ? chunk : g.nz - z;
            HIPCHK(b, launch_export<T>(g, src, b->staging, z, np, b->stream));
            HIPCHK(b, hipMemcpyAsync(dst[q] + (long long)z * plane_c, b->staging,
                                     (size_t)np * plane_c * sizeof(double), hipMemcpyDeviceToHost,
                                     b->stream));
            HIPCHK(b, hipStreamSynchronize(b->stream));
        }
    }
    return FD6_OK;
}

template <typename T>
int batch_reduce(fd6_batch* b, fd6_reductions* out) {
    for (int i = 0; i < b->n; ++i) {
        const fd6_params& p = b->params[i];
        HIPCHK(b, launch_reduce<T>(b->geom[i], fields_of<T>(b->st[b->parity][i].data()),
                                   b->partials, b->results + (size_t)i * kReduceSlots,
                                   p.dx * p.dy * p.dz, b->stream));
    }
    std::vector<double> h((size_t)b->n * kReduceSlots);
    HIPCHK(b, hipMemcpyAsync(h.data(), b->results, h.size() * sizeof(double),
                             hipMemcpyDeviceToHost, b->stream));
    HIPCHK(b, hipStreamSynchronize(b->stream));
    bool bad = false;
    for (int i = 0; i < b->n; ++i) {
        const double* r = &h[(size_t)i * kReduceSlots];
        out[i].mass = r[0];
        out[i].kinetic_energy = r[1];
        out[i].sum_lnrho = r[2];
        out[i].umax = r[3];
        out[i].nonfinite = (int64_t)r[4];
        bad = bad || out[i].nonfinite > 0;
    }
    return bad ? FD6_ENONFINITE : FD6_OK;
}


// ---- ensemble autotuner ----------------------------------------------------
// Candidate z-chunk lengths (0: whole boxes), warm-up and timed steps per
// trial, and passes over the candidates (a candidate's time is its fastest
// trial).  After a change of schedule the step time takes 10-20 steps to
// settle (the first steps of the 64-box ensemble run up to 15% slower), so a
// trial warms up for 10 steps; the passes interleave the candidates, so a
// slower clock at one moment does not decide between schedules a few percent
// apart.
constexpr int kBatchTuneChunks[] = {0, 32, 48, 64, kBatchBalanced, kBatchPacked};
constexpr int kBatchTuneWarmup = 10;
constexpr int kBatchTuneSteps = 8;
constexpr int kBatchTunePasses = 2;

// Two timing events, destroyed with the scope.
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t create() {
        hipError_t e = hipEventCreate(&a);
        return e != hipSuccess ? e : hipEventCreate(&b);
    }
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Cache key of an ensemble: device name, precision, layout, box count and a
// 64-bit FNV-1a hash of the box shapes (one token, no spaces).
std::string batch_tune_key(const fd6_batch* b) {
    int dev = 0;
    hipDeviceProp_t prop{};
    std::string name = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        name = prop.name;
    for (char& c : name)
        if (c == ' ' || c == '\t') c = '_';
    uint64_t h = 1469598103934665603ull;
    for (const fd6_desc& d : b->desc)
        for (int v : {d.nx, d.ny, d.nz}) {
            for (int k = 0; k < 4; ++k) {
                h ^= (uint64_t)((v >> (8 * k)) & 0xff);
                h *= 1099511628211ull;
            }
        }
    char buf[96];
    snprintf(buf, sizeof buf, "|p%d|%s|n%d|%016llx", b->precision, b->aos ? "aos" : "soa", b->n,
             (unsigned long long)h);
    return name + buf;
}

// Cache key of a single box: device name, grid, precision, method, layout.
std::string box_tune_key(const fd6_box* b) {
    int dev = 0;
    hipDeviceProp_t prop{};
    std::string name = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        name = prop.name;
    for (char& c : name)
        if (c == ' ' || c == '\t') c = '_';
    char buf[128];
    snprintf(buf, sizeof buf, "|%dx%dx%d|p%d|v%d|%s", b->desc.nx, b->desc.ny, b->desc.nz,
             b->desc.precision, b->desc.variant, b->geom.vs == 4 ? "aos" : "soa");
    return name + buf;
}

constexpr int kBoxTuneSteps = 2;

// Cache file: one "key tile zchunk" line per box or ensemble; the last match wins.
bool read_tune_cache(const char* path, const std::string& key, int* tile, int* zchunk) {
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char k[512];
    int t = 0, z = 0;
    bool found = false;
    while (fscanf(f, "%511s %d %d", k, &t, &z) == 3)
        if (key == k) *tile = t, *zchunk = z, found = true;
    fclose(f);
    return found;
}

void write_tune_cache(const char* path, const std::string& key, int tile, int zchunk) {
    FILE* f = fopen(path, "a");
    if (!f) return;  // the cache is an optimisation only
    fprintf(f, "%s %d %d\n", key.c_str(), tile, zchunk);
    fclose(f);
}

}  // namespace

extern "C" {

int fd6_abi_version(void) { return FD6_ABI_VERSION; }

const char* fd6_status_string(int s) {
    switch (s) {
    case FD6_OK: return "ok";
    case FD6_EINVAL: return "invalid argument";
    case FD6_ESTATE: return "invalid state (set params and init fields first)";
    case FD6_ENOMEM: return "workspace too small";
    case FD6_EHIP: return "HIP error";
    case FD6_ENONFINITE: return "non-finite values in the state";
    case FD6_EUNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
    }
}

int fd6_workspace_bytes(const fd6_desc* desc, size_t* bytes) {
    if (!bytes) return FD6_EINVAL;
    Plan p;
    int rc = make_plan(desc, &p);
    if (rc) return rc;
    *bytes = p.total;
    return FD6_OK;
}

int fd6_create(const fd6_desc* desc, void* d_ws, size_t bytes, void* stream, fd6_box** out) {
    if (!out || !d_ws) return FD6_EINVAL;
    Plan p;
    int rc = make_plan(desc, &p);
    if (rc) return rc;
    if (((uintptr_t)d_ws) % kAlign != 0) return FD6_EINVAL;
    if (bytes < p.total) return FD6_ENOMEM;
    return guarded((fd6_box*)nullptr, [&]() -> int {
        fd6_box* b = new fd6_box();
        b->desc = *desc;
        // the fastest shapes at 512^3: 64 x 8 for FP32 state, 32 x 8 for FP64
        // (whose 512-thread shapes spill), both two planes ahead
        b->tile = desc->precision == FD6_FP64 ? 8 : 6;
        b->geom = p.g;
        b->stream = static_cast<hipStream_t>(stream);
        b->ws = static_cast<char*>(d_ws);
        b->ws_bytes = bytes;
        b->tsize = p.tsize;
        b->wsize = p.wsize;
        for (int s = 0; s < 2; ++s)
            for (int q = 0; q < 4; ++q) b->state[s][q] = b->ws + p.off_state[s][q];
        for (int q = 0; q < 4; ++q) b->w[q] = b->ws + p.off_w[q];
        b->div = b->ws + p.off_div;
        b->partials = reinterpret_cast<double*>(b->ws + p.off_partials);
        b->result = reinterpret_cast<double*>(b->ws + p.off_result);
        b->force_dev = b->ws + p.off_force;
        b->force_tab = b->ws + p.off_force + kAlign;
        b->staging = reinterpret_cast<double*>(b->ws + p.off_staging);
        b->staging_elems = p.staging_elems;
        *out = b;
        return FD6_OK;
    });
}

int fd6_destroy(fd6_box* b) {
    delete b;
    return FD6_OK;
}

int fd6_set_stream(fd6_box* b, void* stream) {
    if (!b) return FD6_EINVAL;
    b->stream = static_cast<hipStream_t>(stream);
    return FD6_OK;
}

int fd6_set_params(fd6_box* b, const fd6_params* p) {
    if (!b || !p) return FD6_EINVAL;
    if (!finite_nonneg(p->nu) || !finite_nonneg(p->cs) || !finite_pos(p->dx) ||
        !finite_pos(p->dy) || !finite_pos(p->dz) || !finite_pos(p->dt))
        return FD6_EINVAL;
    b->params = *p;
    b->have_params = true;
    b->drop_graphs();         // coefficients are baked into captured steps
    b->force_dirty = true;    // the force amplitude depends on cs and dt
    return FD6_OK;
}

int fd6_set_forcing(fd6_box* b, const fd6_forcing* f) {
    if (!b) return FD6_EINVAL;
    if (!f) {
        if (b->force_on) b->drop_graphs();  // the captured steps add the force
        b->force_on = false;
        return FD6_OK;
    }
    const double v[8] = {f->kx, f->ky, f->kz, f->ex, f->ey, f->ez, f->f0, f->phase};
    for (double x : v)
        if (!std::isfinite(x)) return FD6_EINVAL;
    const double kk2 = f->kx * f->kx + f->ky * f->ky + f->kz * f->kz;
    const double ee = f->ex * f->ex + f->ey * f->ey + f->ez * f->ez;
    const double ke = f->kx * f->ex + f->ky * f->ey + f->kz * f->ez;
    if (!(kk2 > 0.0) || std::fabs(ee - 1.0) > 1e-6 || !(kk2 - ke * ke > 1e-12 * kk2) ||
        f->f0 < 0.0)
        return FD6_EINVAL;
    if (!b->force_on) b->drop_graphs();
    b->force = *f;
    b->force_on = true;
    b->force_dirty = true;
    return FD6_OK;
}

int fd6_init_fields(fd6_box* b, const double* lnrho, const double* ux, const double* uy,
                    const double* uz) {
    if (!b || !lnrho || !ux || !uy || !uz) return FD6_EINVAL;
    return guarded(b, [&]() -> int {
        const double* src[4] = {lnrho, ux, uy, uz};
        b->cur = 0;
        b->ghosts_ok[0] = b->ghosts_ok[1] = false;
        int rc = dispatch(b, [&](auto* t, auto*) -> int {
            using T = std::remove_pointer_t<decltype(t)>;
            return import_host<T>(b, src);
        });
        if (rc) return rc;
        rc = reset_w(b);
        if (rc) return rc;
        HIPCHK(b, hipStreamSynchronize(b->stream));
        b->have_fields = true;
        return FD6_OK;
    });
}

int fd6_init_fields_device(fd6_box* b, const double* lnrho, const double* ux, const double* uy,
                           const double* uz) {
    if (!b || !lnrho || !ux || !uy || !uz) return FD6_EINVAL;
    return guarded(b, [&]() -> int {
        const double* src[4] = {lnrho, ux, uy, uz};
        b->cur = 0;
        b->ghosts_ok[0] = b->ghosts_ok[1] = false;
        int rc = dispatch(b, [&](auto* t, auto*) -> int {
            using T = std::remove_pointer_t<decltype(t)>;
            return import_device<T>(b, src);
        });
        if (rc) return rc;
        rc = reset_w(b);
        if (rc) return rc;
        b->have_fields = true;
        return FD6_OK;
    });
}

int fd6_rk3_step(fd6_box* b, int32_t nsteps) {
    if (!b || nsteps < 0) return FD6_EINVAL;
    if (!ready(b)) return FD6_ESTATE;
    return guarded(b, [&]() -> int {
        return dispatch(b, [&](auto* t, auto* tw) -> int {
            using T = std::remove_pointer_t<decltype(t)>;
            using TW = std::remove_pointer_t<decltype(tw)>;
            return do_steps<T, TW>(b, nsteps);
        });
    });
}

int fd6_rk3_step_reduce(fd6_box* b, int32_t nsteps, double* d_out5) {
    if (!b || nsteps < 1 || !d_out5) return FD6_EINVAL;
    if (!ready(b)) return FD6_ESTATE;
    return guarded(b, [&]() -> int {
        return dispatch(b, [&](auto* t, auto* tw) -> int {
            using T = std::remove_pointer_t<decltype(t)>;
            using TW = std::remove_pointer_t<decltype(tw)>;
            return do_steps<T, TW>(b, nsteps, d_out5);
        });
    });
}

int fd6_get_fields(fd6_box* b, double* lnrho, double* ux, double* uy, double* uz) {
    if (!b || !lnrho || !ux || !uy || !uz) return FD6_EINVAL;
    if (!b->have_fields) return FD6_ESTATE;
    return guarded(b, [&]() -> int {
        double* dst[4] = {lnrho, ux, uy, uz};
        return dispatch(b, [&](auto* t, auto*) -> int {
            using T = std::remove_pointer_t<decltype(t)>;
            return export_host<T>(b, dst);
        });
    });
}

int fd6_get_fields_device(fd6_box* b, double* lnrho, double* ux, double* uy, double* uz) {
    if (!b || !lnrho || !ux || !uy || !uz) return FD6_EINVAL;
    if (!b->have_fields) return FD6_ESTATE;
    return guarded(b, [&]() -> int {
        double* dst[4] = {lnrho, ux, uy, uz};
        return dispatch(b, [&](auto* t, auto*) -> int {
            using T = std::remove_pointer_t<decltype(t)>;
            return export_device<T>(b, dst);
        });
    });
}

int fd6_reduce(fd6_box* b, fd6_reductions* out) {
    if (!b || !out) return FD6_EINVAL;
    if (!ready(b)) return FD6_ESTATE;
    return guarded(b, [&]() -> int {
        return dispatch(b, [&](auto* t, auto*) -> int {
            using T = std::remove_pointer_t<decltype(t)>;
            return do_reduce<T>(b, out);
        });
    });
}

int fd6_reduce_device(fd6_box* b, double* d_out5) {
    if (!b || !d_out5) return FD6_EINVAL;
    if (!ready(b)) return FD6_ESTATE;
    return guarded(b, [&]() -> int {
        return dispatch(b, [&](auto* t, auto*) -> int {
            using T = std::remove_pointer_t<decltype(t)>;
            return do_reduce_device<T>(b, d_out5);
        });
    });
}

int fd6_set_timing(fd6_box* b, int enable) {
    if (!b) return FD6_EINVAL;
    for (auto& p : b->ev_kernel) b->ev_pool.push_back(p.first), b->ev_pool.push_back(p.second);
    for (auto& p : b->ev_ghost) b->ev_pool.push_back(p.first), b->ev_pool.push_back(p.second);
    b->ev_kernel.clear();
    b->ev_ghost.clear();
    b->timing = enable != 0;
    return FD6_OK;
}

int fd6_get_timing(fd6_box* b, double* kernel_ms, int64_t* kernel_launches, double* ghost_ms,
                   int64_t* ghost_launches) {
    if (!b || !kernel_ms || !kernel_launches || !ghost_ms || !ghost_launches) return FD6_EINVAL;
    return guarded(b, [&]() -> int {
        HIPCHK(b, hipStreamSynchronize(b->stream));
        double tk = 0.0, tg = 0.0;
        for (auto& p : b->ev_kernel) {
            float ms = 0.f;
            HIPCHK(b, hipEventElapsedTime(&ms, p.first, p.second));
            tk += ms;
        }
        for (auto& p : b->ev_ghost) {
            float ms = 0.f;
            HIPCHK(b, hipEventElapsedTime(&ms, p.first, p.second));
            tg += ms;
        }
        *kernel_ms = tk;
        *kernel_launches = (int64_t)b->ev_kernel.size();
        *ghost_ms = tg;
        *ghost_launches = (int64_t)b->ev_ghost.size();
        return FD6_OK;
    });
}

int fd6_rhs(fd6_box* b, double* r0, double* r1, double* r2, double* r3) {
    if (!b || !r0 || !r1 || !r2 || !r3) return FD6_EINVAL;
    if (!ready(b)) return FD6_ESTATE;
    return guarded(b, [&]() -> int {
        double* out[4] = {r0, r1, r2, r3};
        return dispatch(b, [&](auto* t, auto* tw) -> int {
            using T = std::remove_pointer_t<decltype(t)>;
            using TW = std::remove_pointer_t<decltype(tw)>;
            return do_rhs<T, TW>(b, out);
        });
    });
}

const char* fd6_last_error(const fd6_box* b) { return b ? b->err.c_str() : ""; }

// Kernel selection for the 55-point substep (tuning hook; 0 = direct
// one-thread-per-point kernel, 1.. = z-sweep tile shapes).
int fd6_set_tile(fd6_box* b, int32_t tile) {
    if (!b || tile < 0 || tile >= substep55_tile_count()) return FD6_EINVAL;
    if (b->geom.vs == 4 && !substep55_aos_tile_ok(tile)) return FD6_EUNSUPPORTED;
    if (tile != b->tile) b->drop_graphs();
    b->tile = tile;
    return FD6_OK;
}

int fd6_set_fused_substeps(fd6_box* b, int32_t enable) {
    if (!b) return FD6_EINVAL;
    if (enable && (b->desc.precision != FD6_FP32 || b->desc.variant != FD6_55P))
        return FD6_EUNSUPPORTED;
    if ((enable != 0) != b->fused12) b->drop_graphs();
    b->fused12 = enable != 0;
    return FD6_OK;
}

int fd6_set_graph(fd6_box* b, int32_t enable) {
    if (!b) return FD6_EINVAL;
    b->use_graph = enable != 0;
    if (!b->use_graph) b->drop_graphs();
    return FD6_OK;
}

int fd6_tile_count(void) { return substep55_tile_count(); }

int fd6_set_zchunk(fd6_box* b, int32_t zchunk) {
    if (!b || zchunk < 0) return FD6_EINVAL;
    if (zchunk != b->zchunk) b->drop_graphs();
    b->zchunk = zchunk;
    return FD6_OK;
}

int fd6_get_schedule(const fd6_box* b, int32_t* tile, int32_t* zchunk) {
    if (!b || !tile || !zchunk) return FD6_EINVAL;
    *tile = b->tile;
    *zchunk = b->zchunk;
    return FD6_OK;
}

int fd6_tune(fd6_box* b, const char* cache_path) {
    if (!b) return FD6_EINVAL;
    if (!ready(b)) return FD6_ESTATE;
    return guarded(b, [&]() -> int {
        const std::string key = box_tune_key(b);
        int tile = 0, zchunk = 0;
        b->tune_log.clear();
        if (cache_path && read_tune_cache(cache_path, key, &tile, &zchunk) &&
            fd6_set_tile(b, tile) == FD6_OK && fd6_set_zchunk(b, zchunk) == FD6_OK)
            return FD6_OK;
        return dispatch(b, [&](auto* t, auto* tw) -> int {
            using T = std::remove_pointer_t<decltype(t)>;
            using TW = std::remove_pointer_t<decltype(tw)>;
            EventPair ev;
            HIPCHK(b, ev.create());
            const bool timing = b->timing;
            b->timing = false;
            // ms per reducing step of one schedule (one warm-up step first)
            auto trial = [&](int cand, int zc, float* ms) -> int {
                if (cand != b->tile || zc != b->zchunk) b->drop_graphs();
                b->tile = cand;
                b->zchunk = zc;
                int rc = do_steps<T, TW>(b, 1, b->result);
                if (rc) return rc;
                HIPCHK(b, hipEventRecord(ev.a, b->stream));
                if ((rc = do_steps<T, TW>(b, kBoxTuneSteps, b->result)) != FD6_OK) return rc;
                HIPCHK(b, hipEventRecord(ev.b, b->stream));
                HIPCHK(b, hipEventSynchronize(ev.b));
                HIPCHK(b, hipEventElapsedTime(ms, ev.a, ev.b));
                *ms /= kBoxTuneSteps;
                b->tune_log.push_back(fd6_box::TuneTrial{cand, zc, *ms});
                return FD6_OK;
            };
            int rc = FD6_OK, best_tile = b->tile, best_zc = b->zchunk;
            float best_ms = -1.0f, ms = 0.0f;
            for (int cand = 1; cand < substep55_tile_count() && rc == FD6_OK; ++cand) {
                if (b->geom.vs == 4 && !substep55_aos_tile_ok(cand)) continue;
                if ((rc = trial(cand, 0, &ms)) == FD6_OK && (best_ms < 0.0f || ms < best_ms))
                    best_ms = ms, best_tile = cand, best_zc = 0;
            }
            // then explicit chunk lengths for that shape, whole columns included
            std::vector<int> chunks;
            for (int zc : {64, 128, 256})
                if (zc < b->desc.nz) chunks.push_back(zc);
            chunks.push_back(b->desc.nz);
            for (int zc : chunks) {
                if (rc != FD6_OK) break;
                if ((rc = trial(best_tile, zc, &ms)) == FD6_OK && ms < best_ms)
                    best_ms = ms, best_zc = zc;
            }
            b->timing = timing;
            if (best_tile != b->tile || best_zc != b->zchunk) b->drop_graphs();
            b->tile = best_tile;
            b->zchunk = best_zc;
            if (rc == FD6_OK && cache_path) write_tune_cache(cache_path, key, best_tile, best_zc);
            return rc;
        });
    });
}

int fd6_get_tune_log(const fd6_box* b, int32_t* tiles, int32_t* zchunks, float* ms,
                     int32_t cap, int32_t* n) {
    if (!b || !n || cap < 0 || (cap > 0 && (!tiles || !zchunks || !ms))) return FD6_EINVAL;
    const int32_t total = (int32_t)b->tune_log.size();
    for (int32_t i = 0; i < total && i < cap; ++i) {
        tiles[i] = b->tune_log[i].tile;
        zchunks[i] = b->tune_log[i].zchunk;
        ms[i] = b->tune_log[i].ms;
    }
    *n = total;
    return FD6_OK;
}

int fd6_batch_workspace_bytes(int32_t n, const fd6_desc* descs, size_t* bytes) {
    if (!bytes) return FD6_EINVAL;
    BatchPlan bp;
    int rc = make_batch_plan(n, descs, &bp);
    if (rc) return rc;
    *bytes = bp.total;
    return FD6_OK;
}

int fd6_batch_create(int32_t n, const fd6_desc* descs, void* d_ws, size_t bytes, void* stream,
                     fd6_batch** out) {
    if (!out || !d_ws) return FD6_EINVAL;
    BatchPlan bp;
    int rc = make_batch_plan(n, descs, &bp);
    if (rc) return rc;
    if (((uintptr_t)d_ws) % kAlign != 0) return FD6_EINVAL;
    if (bytes < bp.total) return FD6_ENOMEM;
    return guarded((fd6_batch*)nullptr, [&]() -> int {
        fd6_batch* b = new fd6_batch();
        b->n = n;
        b->precision = descs[0].precision;
        b->aos = descs[0].flags == FD6_LAYOUT_AOS;
        b->stream = static_cast<hipStream_t>(stream);
        b->ws = static_cast<char*>(d_ws);
        b->ws_bytes = bytes;
        b->desc.assign(descs, descs + n);
        b->geom.resize(n);
        b->params.resize(n);
        b->have_fields.assign(n, false);
        b->st[0].resize(n);
        b->st[1].resize(n);
        b->w.resize(n);
        for (int i = 0; i < n; ++i) {
            const Plan& p = bp.box[i];
            b->geom[i] = p.g;
            char* base = b->ws + bp.base[i];
            for (int s = 0; s < 2; ++s)
                for (int q = 0; q < 4; ++q) b->st[s][i][q] = base + p.off_state[s][q];
            for (int q = 0; q < 4; ++q) b->w[i][q] = base + p.off_w[q];
        }
        b->tsize = bp.box[0].tsize;
        b->wsize = bp.box[0].wsize;
        b->boxes_dev = b->ws + bp.off_boxes;
        b->box_bytes = bp.box_bytes;
        b->items_dev = reinterpret_cast<BatchItem*>(b->ws + bp.off_items);
        b->wg_first_dev = reinterpret_cast<int*>(b->ws + bp.off_wg);
        b->items_cap = bp.items_cap;
        b->partials = reinterpret_cast<double*>(b->ws + bp.off_partials);
        b->results = reinterpret_cast<double*>(b->ws + bp.off_results);
        b->staging = reinterpret_cast<double*>(b->ws + bp.off_staging);
        b->staging_elems = bp.staging_elems;
        *out = b;
        return FD6_OK;
    });
}

int fd6_batch_destroy(fd6_batch* b) {
    delete b;
    return FD6_OK;
}

int fd6_batch_set_params(fd6_batch* b, const fd6_params* per_box) {
    if (!b || !per_box) return FD6_EINVAL;
    for (int i = 0; i < b->n; ++i) {
        const fd6_params* p = &per_box[i];
        if (!finite_nonneg(p->nu) || !finite_nonneg(p->cs) || !finite_pos(p->dx) ||
            !finite_pos(p->dy) || !finite_pos(p->dz) || !finite_pos(p->dt))
            return FD6_EINVAL;
    }
    return guarded(b, [&]() -> int {
        b->params.assign(per_box, per_box + b->n);
        b->have_params = true;
        return batch_dispatch(b, [&](auto* t, auto* tw) -> int {
            using T = std::remove_pointer_t<decltype(t)>;
            using TW = std::remove_pointer_t<decltype(tw)>;
            return upload_boxes<T, TW>(b);
        });
    });
}

int fd6_batch_init_fields(fd6_batch* b, int32_t box, const double* lnrho, const double* ux,
                          const double* uy, const double* uz) {
    if (!b || box < 0 || box >= b->n || !lnrho || !ux || !uy || !uz) return FD6_EINVAL;
    return guarded(b, [&]() -> int {
        const double* src[4] = {lnrho, ux, uy, uz};
        int rc = batch_dispatch(b, [&](auto* t, auto* tw) -> int {
            using T = std::remove_pointer_t<decltype(t)>;
            using TW = std::remove_pointer_t<decltype(tw)>;
            int r = batch_import<T>(b, box, src);
            if (r) return r;
            HIPCHK(b, launch_zero_w<TW>(b->geom[box], fields_of<TW>(b->w[box].data()), b->stream));
            HIPCHK(b, hipStreamSynchronize(b->stream));
            return FD6_OK;
        });
        if (rc) return rc;
        b->have_fields[box] = true;
        return FD6_OK;
    });
}

int fd6_batch_set_schedule(fd6_batch* b, int32_t tile, int32_t zchunk) {
    int tx, ty;
    if (!b || !batch_zchunk_ok(zchunk) || substep55_tile_dims(tile, &tx, &ty))
        return FD6_EINVAL;
    if (b->aos && !substep55_aos_tile_ok(tile)) return FD6_EUNSUPPORTED;
    return guarded(b, [&]() -> int {
        return batch_dispatch(b, [&](auto* t, auto* tw) -> int {
            using T = std::remove_pointer_t<decltype(t)>;
            using TW = std::remove_pointer_t<decltype(tw)>;
            return build_items<T, TW>(b, tile, zchunk);
        });
    });
}

int fd6_batch_set_graph(fd6_batch* b, int32_t enable) {
    if (!b) return FD6_EINVAL;
    b->use_graph = enable != 0;
    return FD6_OK;
}

int fd6_batch_step(fd6_batch* b, int32_t nsteps) {
    if (!b || nsteps < 0) return FD6_EINVAL;
    if (!b->have_params) return FD6_ESTATE;
    for (int i = 0; i < b->n; ++i)
        if (!b->have_fields[i]) return FD6_ESTATE;
    return guarded(b, [&]() -> int {
        return batch_dispatch(b, [&](auto* t, auto* tw) -> int {
            using T = std::remove_pointer_t<decltype(t)>;
            using TW = std::remove_pointer_t<decltype(tw)>;
            return batch_steps<T, TW>(b, nsteps);
        });
    });
}

int fd6_batch_get_schedule(const fd6_batch* b, int32_t* tile, int32_t* zchunk) {
    if (!b || !tile || !zchunk) return FD6_EINVAL;
    *tile = b->tile;
    *zchunk = b->zchunk;
    return FD6_OK;
}

int fd6_batch_tune(fd6_batch* b, const char* cache_path) {
    if (!b) return FD6_EINVAL;
    if (!b->have_params) return FD6_ESTATE;
    for (int i = 0; i < b->n; ++i)
        if (!b->have_fields[i]) return FD6_ESTATE;
    return guarded(b, [&]() -> int {
        const std::string key = batch_tune_key(b);
        int tile = 0, zchunk = 0;
        if (cache_path && read_tune_cache(cache_path, key, &tile, &zchunk) &&
            fd6_batch_set_schedule(b, tile, zchunk) == FD6_OK)
            return FD6_OK;
        return batch_dispatch(b, [&](auto* t, auto* tw) -> int {
            using T = std::remove_pointer_t<decltype(t)>;
            using TW = std::remove_pointer_t<decltype(tw)>;
            EventPair ev;
            HIPCHK(b, ev.create());
            float best_ms = -1.0f;
            const int old_tile = b->tile, old_zc = b->zchunk;
            int best_tile = old_tile, best_zc = old_zc;
            // time of one candidate schedule (warm-up steps, the first of
            // which captures its graphs, then kBatchTuneSteps timed steps)
            auto trial = [&](int cand, int zc, float* ms) -> int {
                int r = build_items<T, TW>(b, cand, zc);
                if (r == FD6_OK) r = batch_steps<T, TW>(b, kBatchTuneWarmup);
                if (r) return r;
                HIPCHK(b, hipEventRecord(ev.a, b->stream));
                if ((r = batch_steps<T, TW>(b, kBatchTuneSteps)) != FD6_OK) return r;
                HIPCHK(b, hipEventRecord(ev.b, b->stream));
                HIPCHK(b, hipEventSynchronize(ev.b));
                HIPCHK(b, hipEventElapsedTime(ms, ev.a, ev.b));
                return FD6_OK;
            };
            std::vector<std::pair<int, int>> cands;  // (shape, z-chunk)
            for (int cand = 1; cand < substep55_tile_count(); ++cand) {
                int tx, ty;
                if (substep55_tile_dims(cand, &tx, &ty) != 0) continue;
                if (b->aos && !substep55_aos_tile_ok(cand)) continue;
                for (int zc : kBatchTuneChunks) cands.emplace_back(cand, zc);
            }
            std::vector<float> fastest(cands.size(), -1.0f);
            int rc = FD6_OK;
            for (int pass = 0; pass < kBatchTunePasses && rc == FD6_OK; ++pass)
                for (size_t k = 0; k < cands.size(); ++k) {
                    float ms = 0.0f;
                    if ((rc = trial(cands[k].first, cands[k].second, &ms)) != FD6_OK) break;
                    if (fastest[k] < 0.0f || ms < fastest[k]) fastest[k] = ms;
                }
            for (size_t k = 0; k < cands.size() && rc == FD6_OK; ++k)
                if (best_ms < 0.0f || fastest[k] < best_ms)
                    best_ms = fastest[k], best_tile = cands[k].first, best_zc = cands[k].second;
            if (rc != FD6_OK) {
                // a failed trial leaves the schedule that was in force before
                (void)build_items<T, TW>(b, old_tile, old_zc);
                return rc;
            }
            rc = build_items<T, TW>(b, best_tile, best_zc);
            if (rc == FD6_OK && cache_path) write_tune_cache(cache_path, key, best_tile, best_zc);
            return rc;
        });
    });
}

int fd6_batch_get_fields(fd6_batch* b, int32_t box, double* lnrho, double* ux, double* uy,
                         double* uz) {
    if (!b || box < 0 || box >= b->n || !lnrho || !ux || !uy || !uz) return FD6_EINVAL;
    if (!b->have_fields[box]) return FD6_ESTATE;
    return guarded(b, [&]() -> int {
        double* dst[4] = {lnrho, ux, uy, uz};
        return batch_dispatch(b, [&](auto* t, auto*) -> int {
            using T = std::remove_pointer_t<decltype(t)>;
            return batch_export<T>(b, box, dst);
        });
    });
}

int fd6_batch_reduce(fd6_batch* b, fd6_reductions* per_box) {
    if (!b || !per_box) return FD6_EINVAL;
    if (!b->have_params) return FD6_ESTATE;
    for (int i = 0; i < b->n; ++i)
        if (!b->have_fields[i]) return FD6_ESTATE;
    return guarded(b, [&]() -> int {
        return batch_dispatch(b, [&](auto* t, auto*) -> int {
            using T = std::remove_pointer_t<decltype(t)>;
            return batch_reduce<T>(b, per_box);
        });
    });
}

const char* fd6_batch_last_error(const fd6_batch* b) { return b ? b->err.c_str() : ""; }


}  // extern "C"

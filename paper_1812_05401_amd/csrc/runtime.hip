// Host runtime and C ABI of the VP-LBM library (see include/vplbm.h).
//
// A simulation owns two population buffers (A/B ping-pong: a step reads one and writes the other,
// so there is no read-after-write hazard inside a step), a body-id plane, a small body table and
// a ring of per-step FP64 observables.  Steps are replayed in chunks from captured HIP graphs
// (one per buffer parity) so that the host is not on the per-step path; the step counter lives on
// the device and the graph ends with a kernel that advances it.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <string>
#include <unordered_set>

#include "internal.hpp"
#include "kernels.hpp"
#include "static_scratch.hpp"
#include "step_plan.hpp"
#include "vplbm.h"

using namespace vplbm;

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace vplbm {

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}



void host_log(const char *fmt, ...)
{
    const char *e = getenv("VPLBM_LOG");
    if (!e || atoi(e) < 1) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    fprintf(stderr, "[vplbm] %s\n", buf);
}

static_assert(int(kF64) == int(VPLBM_F64) && int(kF32) == int(VPLBM_F32) &&
                  int(kF16S) == int(VPLBM_F16S) && int(kBF16S) == int(VPLBM_BF16S) &&
                  int(kF32D) == int(VPLBM_F32D) && int(kF16SR) == int(VPLBM_F16SR) &&
                  int(kBF16SR) == int(VPLBM_BF16SR),
              "device storage ids follow the ABI");

int elem_bytes(int storage)
{
    switch (storage) {
    case VPLBM_F64: return 8;
    case VPLBM_F32:
    case VPLBM_F32D: return 4;
    case VPLBM_F16S:
    case VPLBM_BF16S:
    case VPLBM_F16SR:
    case VPLBM_BF16SR: return 2;
    default: return 0;
    }
}

}  // namespace vplbm

namespace {

// Steps per captured graph replay.  128 (measured): 1.2% faster than 32 on the cache-resident
// 2048 x 512 lattice, where the step-counter node and the gap between replays are a visible share
// of a 22 us launch pair; no change on large lattices.  Calls of fewer steps are launched
// directly.
int graph_chunk()
{
    int k = 128;
    if (const char *e = getenv("VPLBM_GRAPH_STEPS")) k = atoi(e);
    if (k < 0) k = 0;
    return k & ~1;   // even: a replay is whole two-step launches where those apply
}

}  // namespace

struct vplbm_sim_s {
    vplbm_config cfg{};
    Geom g{};
    TileShape ts{};
    int storage = 0;
    size_t buf_bytes = 0;
    void *buf[2] = {nullptr, nullptr};
    int cur = 0;                         // buffer holding the current post-collision state
    uint8_t *mask = nullptr;
    BodyParams *d_params = nullptr;
    BodyState *d_state = nullptr;
    uint8_t *mask_alt = nullptr;         // moving bodies: mask and body states of the first step of
    BodyState *d_state_alt = nullptr;    //   a two- or three-step launch (mask / d_state take the last)
    uint8_t *mask_alt2 = nullptr;        //   and of the second step of a three-step launch
    BodyState *d_state_alt2 = nullptr;
    BodyParams h_params[kMaxBodies];
    int nbodies = 0;
    bool device_mask = false;
    bool moving = false;
    int env_box[kMaxBodies][4];          // x0, y0, w, h swept by each moving body
    double *ring = nullptr;
    double *acc = nullptr;               // [kAccSets][kSub][kRingWidth] reduction sub-slots
    int ring_len = 0;
    unsigned *status = nullptr;
    long long *t_dev = nullptr;
    double *staging = nullptr;          // dense FP64 host<->device staging
    void *outlet[2] = {nullptr, nullptr}; // convective outlet state per buffer parity
    size_t staging_bytes = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;                      // the device current at create (holds all the memory)
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int graph_flip[2] = {0, 0};          // 1: a replay moves the state to the other buffer
    int graph_k = 0;
    bool two_step = true;                // two steps per launch where the case allows it
    bool three_step = true;              // three where the kernel exists for the case
    int64_t steps = 0;
    bool unstable = false;
    NodeParams params{};
    int nt_store = 0;
    double *snap = nullptr;              // convergence residual: [2][ny*nx] velocity snapshot,
    double *rpart = nullptr;             // then per-workgroup partials and the two sums
    bool have_snap = false;
};

namespace {

// Live handles, so that a NULL, stale or foreign handle is rejected instead of dereferenced.
std::mutex g_live_mu;
std::unordered_set<const void *> g_live;

bool valid(const void *s)
{
    if (!s) return false;
    std::lock_guard<std::mutex> lk(g_live_mu);
    return g_live.count(s) != 0;
}

void track(const void *s, bool live)
{
    std::lock_guard<std::mutex> lk(g_live_mu);
    if (live) g_live.insert(s);
    else g_live.erase(s);
}

StepArgs step_args(vplbm_sim s, int src, int t_off)
{
    StepArgs a{};
    a.src = s->buf[src];
    a.dst = s->buf[src ^ 1];
    a.mask = s->mask;
    a.bodies = s->d_state;
    a.mask2 = s->mask;
    a.bodies2 = s->d_state;
    a.mask3 = s->mask;
    a.bodies3 = s->d_state;
    a.ring = s->ring;
    a.acc = s->acc;
    a.status = s->status;
    a.t_base = s->t_dev;
    a.g = s->g;
    a.outlet.prev = s->outlet[src];
    a.outlet.next = s->outlet[src ^ 1];
    a.outlet.u = s->cfg.u_in_x;
    a.t_off = t_off;
    a.ring_len = s->ring_len;
    a.reduce = s->cfg.reduce;
    a.ntx = s->ts.ntx;
    a.bx_log2 = s->ts.bx_log2;
    a.by = s->ts.by;
    a.rows = s->ts.rows;
    a.nt_store = s->nt_store;
    a.p = s->params;
    return a;
}

// Body states and the swept part of the mask for the n (1 or 2) steps at *t_dev + t_off, ...
// (moving bodies), in one launch: step s into masks[s] / states[s] (the simulation's own, or for
// the first step of a two-step launch the other mask and state array).
hipError_t place_bodies_n(vplbm_sim s, int t_off, int n, hipStream_t st, uint8_t *const *masks,
                          BodyState *const *states)
{
    PlaceArgs a{};
    a.params = s->d_params;
    a.nbodies = s->nbodies;
    a.nsteps = n;
    for (int i = 0; i < n; i++) {
        a.mask[i] = masks[i];
        a.state[i] = states[i];
    }
    a.t_base = s->t_dev;
    a.t_off = t_off;
    a.g = s->g;
    int acc = 0;
    for (int k = 0; k < kMaxBodies; k++) {
        a.box_start[k] = acc;
        const int *b = s->env_box[k];
        const bool use = s->moving && k < s->nbodies && b[2] > 0 && b[3] > 0;
        for (int q = 0; q < 4; q++) a.box[k][q] = use ? b[q] : 0;
        acc += use ? b[2] * b[3] : 0;
    }
    a.box_start[kMaxBodies] = acc;
    return launch_place(a, st);
}

hipError_t place_bodies(vplbm_sim s, int t_off, hipStream_t st)
{
    uint8_t *m[1] = {s->mask};
    BodyState *b[1] = {s->d_state};
    return place_bodies_n(s, t_off, 1, st, m, b);
}

// Convective outlet: the previous-step outlet values start as the current state's last column.
hipError_t reset_outlet(vplbm_sim s)
{
    if (!s->outlet[0]) return hipSuccess;
    return launch_outlet_init(s->storage, step_args(s, s->cur, 0), s->outlet[s->cur], s->stream);
}

// Two steps per launch: moving bodies take a second mask for the first step.
bool two_step_ok(vplbm_sim s)
{
    return s->two_step && (!s->moving || s->mask_alt);
}

// Three steps per launch: binary32 storage, planes below 4 GB (the kernel stores through a 32-bit
// buffer resource); moving bodies take masks of their own for the first two steps.
bool three_step_ok(vplbm_sim s)
{
    return s->three_step && two_step_ok(s) && step3_supported(s->storage) &&
           s->buf_bytes <= 0xFFFFFFFFu && (!s->moving || s->mask_alt2);
}

// Enqueue n steps starting from the state in buf[first_src]: triples of steps in three-step
// launches where the case allows them (unless VPLBM_THREE_STEP=0 turned them off), else pairs in
// two-step launches (unless VPLBM_TWO_STEP=0), and what remains one or two at a time.  Every
// launch moves the state to the other buffer; *flip is the parity of the number of launches.
hipError_t enqueue_steps(vplbm_sim s, int first_src, int n, hipStream_t st, int *flip)
{
    const bool two = two_step_ok(s);
    const bool three = three_step_ok(s);
    int src = first_src;
    int j = 0;
    while (j < n) {
        hipError_t e;
        if (three && n - j >= 3) {
            StepArgs a = step_args(s, src, j);
            if (s->moving) {
                // steps one and two on the other masks, the third on the simulation's own
                uint8_t *m[3] = {s->mask_alt, s->mask_alt2, s->mask};
                BodyState *b[3] = {s->d_state_alt, s->d_state_alt2, s->d_state};
                e = place_bodies_n(s, j, 3, st, m, b);
                if (e != hipSuccess) return e;
                a.mask = s->mask_alt;
                a.bodies = s->d_state_alt;
                a.mask2 = s->mask_alt2;
                a.bodies2 = s->d_state_alt2;
            }
            e = launch_step3(s->storage, a, st);
            j += 3;
        } else if (two && n - j >= 2) {
            StepArgs a = step_args(s, src, j);
            if (s->moving) {
                // the first step on the other mask, the second on the simulation's own: after
                // the launch it holds the last step's bodies, as after one step per launch
                uint8_t *m[2] = {s->mask_alt, s->mask};
                BodyState *b[2] = {s->d_state_alt, s->d_state};
                e = place_bodies_n(s, j, 2, st, m, b);
                if (e != hipSuccess) return e;
                a.mask = s->mask_alt;
                a.bodies = s->d_state_alt;
            }
            e = launch_step2(s->storage, a, st);
            j += 2;
        } else {
            if (s->moving) {
                e = place_bodies(s, j, st);
                if (e != hipSuccess) return e;
            }
            e = launch_step(s->storage, step_args(s, src, j), st);
            j += 1;
        }
        if (e != hipSuccess) return e;
        src ^= 1;
    }
    *flip = src ^ first_src;
    return launch_advance(s->t_dev, n, st);
}

int ensure_graph(vplbm_sim s, int parity)
{
    if (s->graph[parity]) return VPLBM_OK;
    if (!s->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&s->cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = enqueue_steps(s, parity, s->graph_k, s->cap_stream, &s->graph_flip[parity]);
    hipError_t e2 = hipStreamEndCapture(s->cap_stream, &graph);
    if (e != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(VPLBM_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    }
    HIP_TRY(e2);
    e = hipGraphInstantiate(&s->graph[parity], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIP_TRY(e);
    return VPLBM_OK;
}

int ensure_staging(vplbm_sim s, size_t bytes)
{
    if (s->staging_bytes >= bytes) return VPLBM_OK;
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (s->staging) HIP_TRY(hipFree(s->staging));
    s->staging = nullptr;
    s->staging_bytes = 0;
    if (hipMalloc(&s->staging, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(VPLBM_ENOMEM, "cannot allocate %zu bytes of staging memory", bytes);
    }
    s->staging_bytes = bytes;
    return VPLBM_OK;
}

void release(vplbm_sim s)
{
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (int p = 0; p < 2; p++)
        if (s->graph[p]) (void)hipGraphExecDestroy(s->graph[p]);
    void *ptrs[] = {s->buf[0], s->buf[1], s->mask, s->mask_alt, s->mask_alt2, s->d_params, s->d_state,
                    s->d_state_alt, s->d_state_alt2, s->ring, s->acc,
                    s->status, s->t_dev, s->staging, s->outlet[0], s->outlet[1], s->snap, s->rpart};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    if (s->cap_stream) (void)hipStreamDestroy(s->cap_stream);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    track(s, false);
    delete s;
}

}  // namespace

namespace vplbm {

NodeParams node_params(const vplbm_config &c)
{
    NodeParams p{};
    // Relaxation: MRT = rates of Eq. 14 (s_n = 1/tau, s_q from Lambda, Eq. 15); SRT = 1/tau.
    p.sp = 1.0 / c.tau;
    p.sm = c.collision == VPLBM_MRT ? 1.0 / (0.5 + c.lambda / (c.tau - 0.5)) : p.sp;
    p.kp = 1.0 - 0.5 * p.sp;
    p.km = 1.0 - 0.5 * p.sm;
    // Penalization (Eqs. 17-18, dt = 1): k = 1/(1 + 1/(2 eta)) = 2 eta/(2 eta + 1).
    p.k_relax = 2.0 * c.eta / (2.0 * c.eta + 1.0);
    p.c_pen = 1.0 / (c.eta + 0.5);
    p.uin_x = c.u_in_x;
    p.uin_y = c.u_in_y;
    return p;
}

int check_config(const vplbm_config *c)
{
    if (!c) return fail(VPLBM_EINVAL, "config is NULL");
    if (c->abi_version != VPLBM_ABI_VERSION)
        return fail(VPLBM_EINVAL, "abi_version %u, library is %d", c->abi_version, VPLBM_ABI_VERSION);
    if (c->nx < 3 || c->ny < 3) return fail(VPLBM_EINVAL, "lattice %dx%d: both sides must be >= 3", c->nx, c->ny);
    const long long pitch = (c->nx + 63) / 64 * 64;
    if (pitch * (long long)c->ny * 9 + 64 * 9 >= (1LL << 31))
        return fail(VPLBM_EINVAL, "lattice %dx%d too large for 32-bit plane offsets", c->nx, c->ny);
    if (c->collision != VPLBM_SRT && c->collision != VPLBM_MRT)
        return fail(VPLBM_EINVAL, "unknown collision %d", c->collision);
    if (!elem_bytes(c->storage)) return fail(VPLBM_EINVAL, "unknown storage %d", c->storage);
    if (!(c->tau > 0.5) || !isfinite(c->tau)) return fail(VPLBM_EINVAL, "tau must be > 1/2 (got %g)", c->tau);
    if (c->collision == VPLBM_MRT && (!(c->lambda > 0) || !isfinite(c->lambda)))
        return fail(VPLBM_EINVAL, "MRT needs Lambda > 0 (got %g)", c->lambda);
    if (!(c->eta > 0) || !isfinite(c->eta)) return fail(VPLBM_EINVAL, "eta must be > 0 (got %g)", c->eta);
    if (!(c->rho0 > 0) || !isfinite(c->rho0)) return fail(VPLBM_EINVAL, "rho0 must be > 0");
    if (!isfinite(c->ux0) || !isfinite(c->uy0)) return fail(VPLBM_EINVAL, "initial velocity must be finite");
    const bool xper = c->bc_xlo == VPLBM_PERIODIC && c->bc_xhi == VPLBM_PERIODIC;
    const bool xio = c->bc_xlo == VPLBM_VELOCITY && (c->bc_xhi == VPLBM_OUTFLOW || c->bc_xhi == VPLBM_CONVECTIVE);
    const bool yper = c->bc_ylo == VPLBM_PERIODIC && c->bc_yhi == VPLBM_PERIODIC;
    const bool yfs = c->bc_ylo == VPLBM_FREESLIP && c->bc_yhi == VPLBM_FREESLIP;
    if (!(xper || xio))
        return fail(VPLBM_EINVAL, "x edges must be PERIODIC/PERIODIC or VELOCITY/OUTFLOW|CONVECTIVE (got %d/%d)", c->bc_xlo, c->bc_xhi);
    if (!(yper || yfs))
        return fail(VPLBM_EINVAL, "y edges must be PERIODIC/PERIODIC or FREESLIP/FREESLIP (got %d/%d)", c->bc_ylo, c->bc_yhi);
    if (c->bc_xhi == VPLBM_CONVECTIVE && !(c->u_in_x > 0.0))
        return fail(VPLBM_EINVAL, "a convective outlet needs a positive convection speed u_in_x");
    if (xio && !(fabs(c->u_in_x) < 1.0 && isfinite(c->u_in_y)))
        return fail(VPLBM_EINVAL, "inlet velocity must satisfy |u_in_x| < 1");
    if (c->reduce != 0 && c->reduce != 1) return fail(VPLBM_EINVAL, "reduce must be 0 or 1");
    if (c->ring < 0 || c->ring == 1) return fail(VPLBM_EINVAL, "ring must be 0 or >= 2");
    return VPLBM_OK;
}

int check_bodies(const vplbm_body *b, int n)
{
    if (n < 0 || n > VPLBM_MAX_BODIES) return fail(VPLBM_EINVAL, "nbodies %d not in [0, 8]", n);
    if (n > 0 && !b) return fail(VPLBM_EINVAL, "bodies is NULL");
    for (int k = 0; k < n; k++) {
        const vplbm_body &x = b[k];
        if (x.kind < VPLBM_DISK || x.kind > VPLBM_DISK_OUTSIDE) return fail(VPLBM_EINVAL, "body %d: unknown shape %d", k, x.kind);
        const double v[] = {x.cx, x.cy, x.r, x.hx, x.hy, x.ux, x.uy, x.omega, x.ax, x.ay, x.freq};
        for (double d : v)
            if (!isfinite(d)) return fail(VPLBM_EINVAL, "body %d has a non-finite parameter", k);
        if (x.r < 0 || x.hx < 0 || x.hy < 0) return fail(VPLBM_EINVAL, "body %d has a negative size", k);
    }
    return VPLBM_OK;
}

}  // namespace vplbm

extern "C" {

const char *vplbm_last_error(void) { return g_last_error.c_str(); }

int vplbm_bytes_per_update(int32_t storage, int64_t *bytes)
{
    const int e = elem_bytes(storage);
    if (!e || !bytes) return fail(VPLBM_EINVAL, "unknown storage %d or NULL output", storage);
    *bytes = 18LL * e + 1;
    return VPLBM_OK;
}

int vplbm_create(const vplbm_config *cfg, vplbm_sim *out)
{
    if (!out) return fail(VPLBM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_config(cfg);
    if (rc) return rc;
    vplbm_sim s = new vplbm_sim_s();
    s->cfg = *cfg;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return fail(VPLBM_EHIP, "no current device");
    }
    // the allocation-free entry point's scratch on this device (an error is reported by that call)
    if (static_scratch_init() != VPLBM_OK) host_log("static scratch: %s", vplbm_last_error());
    s->storage = cfg->storage;
    s->ring_len = cfg->ring ? cfg->ring : 4096;
    s->graph_k = graph_chunk();
    s->params = node_params(*cfg);

    Geom &g = s->g;
    g.nx = cfg->nx;
    g.ny = cfg->ny;
    g.pitch = (cfg->nx + 63) / 64 * 64;
    g.plane = g.pitch * cfg->ny;
    g.xper = cfg->bc_xlo == VPLBM_PERIODIC;
    g.yper = cfg->bc_ylo == VPLBM_PERIODIC;
    g.inlet = cfg->bc_xlo == VPLBM_VELOCITY;
    s->ts = tile_shape(g.nx, g.ny, elem_bytes(cfg->storage));

    if (cfg->stream) {
        s->stream = (hipStream_t)cfg->stream;
    } else {
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
            delete s;
            return fail(VPLBM_EHIP, "cannot create a stream");
        }
        s->own_stream = true;
    }
    const int eb = elem_bytes(s->storage);
    s->buf_bytes = (size_t)9 * g.plane * eb;
    // Both buffers beyond the 256 MB Infinity Cache: the stores stream past it (measured 6%
    // faster there; inside the cache normal stores keep the next step's reads on chip).
    s->nt_store = 2 * s->buf_bytes > ((size_t)192 << 20) ? 1 : 0;
    if (const char *e = getenv("VPLBM_NT_STORE")) s->nt_store = atoi(e) ? 1 : 0;
    if (const char *e = getenv("VPLBM_TWO_STEP")) s->two_step = atoi(e) != 0;   // 0: one step per launch
    if (const char *e = getenv("VPLBM_THREE_STEP")) s->three_step = atoi(e) != 0; // 0: at most two
    struct { void **p; size_t n; } allocs[] = {
        {&s->buf[0], s->buf_bytes}, {&s->buf[1], s->buf_bytes},
        {(void **)&s->mask, (size_t)g.pitch * g.ny},
        {(void **)&s->d_params, sizeof(BodyParams) * kMaxBodies},
        {(void **)&s->d_state, sizeof(BodyState) * kMaxBodies},
        {(void **)&s->d_state_alt, sizeof(BodyState) * kMaxBodies},
        {(void **)&s->d_state_alt2, sizeof(BodyState) * kMaxBodies},
        {(void **)&s->ring, sizeof(double) * kRingWidth * s->ring_len},
        {(void **)&s->acc, sizeof(double) * kAccSets * kSub * kRingWidth},
        {(void **)&s->status, sizeof(unsigned) * 4},
        {(void **)&s->t_dev, sizeof(long long)},
        {&s->outlet[0], cfg->bc_xhi == VPLBM_CONVECTIVE ? sizeof(double) * 3 * g.ny : 0},
        {&s->outlet[1], cfg->bc_xhi == VPLBM_CONVECTIVE ? sizeof(double) * 3 * g.ny : 0},
    };
    for (auto &a : allocs) {
        if (a.n == 0) continue;
        if (hipMalloc(a.p, a.n) != hipSuccess) {
            (void)hipGetLastError();
            size_t need = a.n;
            release(s);
            return fail(VPLBM_ENOMEM, "cannot allocate %zu bytes of device memory", need);
        }
    }
    hipError_t e = hipMemsetAsync(s->mask, 0, (size_t)g.pitch * g.ny, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_state, 0, sizeof(BodyState) * kMaxBodies, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_state_alt, 0, sizeof(BodyState) * kMaxBodies, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_state_alt2, 0, sizeof(BodyState) * kMaxBodies, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->d_params, 0, sizeof(BodyParams) * kMaxBodies, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->ring, 0, sizeof(double) * kRingWidth * s->ring_len, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->acc, 0, sizeof(double) * kAccSets * kSub * kRingWidth, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->status, 0, sizeof(unsigned) * 4, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->t_dev, 0, sizeof(long long), s->stream);
    // Padding columns and the planes' tails are never read for results; clear them once.
    if (e == hipSuccess) e = hipMemsetAsync(s->buf[0], 0, s->buf_bytes, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->buf[1], 0, s->buf_bytes, s->stream);
    if (e == hipSuccess) e = launch_init(s->storage, step_args(s, 1, 0), nullptr, nullptr, nullptr, cfg->rho0, cfg->ux0, cfg->uy0, s->stream);
    s->cur = 0;
    if (e == hipSuccess) e = reset_outlet(s);
    if (e != hipSuccess) {
        release(s);
        return fail(VPLBM_EHIP, "initialisation failed: %s", hipGetErrorString(e));
    }
    track(s, true);
    *out = s;
    host_log("create %p: %dx%d storage %d collision %d, tiles %dx%d x %d rows, %d planes of %d elements, "
        "non-temporal stores %d, steps per launch %d", (void *)s, g.nx, g.ny, s->storage, cfg->collision,
        1 << s->ts.bx_log2, s->ts.by, s->ts.rows, 9, g.plane, s->nt_store,
        three_step_ok(s) ? 3 : two_step_ok(s) ? 2 : 1);
    return VPLBM_OK;
}

int vplbm_destroy(vplbm_sim s)
{
    if (!s) return VPLBM_OK;
    if (!valid(s)) return fail(VPLBM_EINVAL, "invalid handle");
    host_log("destroy %p after %lld steps", (void *)s, (long long)s->steps);
    release(s);
    return VPLBM_OK;
}

int vplbm_set_mask(vplbm_sim s, const uint8_t *body_id, const vplbm_body *bodies, int32_t nbodies)
{
    if (!valid(s)) return fail(VPLBM_EINVAL, "invalid handle");
    int rc = check_bodies(bodies, nbodies);
    if (rc) return rc;
    bool moving = false;
    for (int k = 0; k < nbodies; k++)
        if (bodies[k].freq != 0.0 && (bodies[k].ax != 0.0 || bodies[k].ay != 0.0)) moving = true;
    if (moving && body_id) return fail(VPLBM_EINVAL, "moving bodies need a device-rasterized mask (body_id = NULL)");
    const Geom &g = s->g;
    if (body_id) {
        const size_t n = (size_t)g.nx * g.ny;
        for (size_t i = 0; i < n; i++)
            if (body_id[i] > nbodies) return fail(VPLBM_EINVAL, "body_id[%zu] = %d but only %d bodies", i, body_id[i], nbodies);
    }
    // The graphs hold pointers only, but moving-body nodes are part of them: rebuild lazily.
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (int p = 0; p < 2; p++)
        if (s->graph[p]) {
            HIP_TRY(hipGraphExecDestroy(s->graph[p]));
            s->graph[p] = nullptr;
        }
    for (int k = 0; k < nbodies; k++) {
        const vplbm_body &b = bodies[k];
        BodyParams &p = s->h_params[k];
        p.kind = b.kind; p.cx = b.cx; p.cy = b.cy; p.r = b.r; p.hx = b.hx; p.hy = b.hy;
        p.ux = b.ux; p.uy = b.uy; p.omega = b.omega; p.ax = b.ax; p.ay = b.ay; p.freq = b.freq;
        // Box swept by a moving body over its whole stroke (+2 nodes of margin).
        int *box = s->env_box[k];
        box[0] = box[1] = box[2] = box[3] = 0;
        const bool mv = b.freq != 0.0 && (b.ax != 0.0 || b.ay != 0.0);
        if (mv) {
            if (b.kind == VPLBM_DISK_OUTSIDE) {
                box[0] = 0; box[1] = 0; box[2] = g.nx; box[3] = g.ny;
            } else {
                const double ex = (b.kind == VPLBM_DISK ? b.r : b.hx) + fabs(b.ax) + 2.0;
                const double ey = (b.kind == VPLBM_DISK ? b.r : b.hy) + fabs(b.ay) + 2.0;
                long x0 = (long)floor(b.cx - ex), x1 = (long)ceil(b.cx + ex);
                long y0 = (long)floor(b.cy - ey), y1 = (long)ceil(b.cy + ey);
                x0 = x0 < 0 ? 0 : x0; y0 = y0 < 0 ? 0 : y0;
                x1 = x1 > g.nx - 1 ? g.nx - 1 : x1; y1 = y1 > g.ny - 1 ? g.ny - 1 : y1;
                if (x1 >= x0 && y1 >= y0) {
                    box[0] = (int)x0; box[1] = (int)y0; box[2] = (int)(x1 - x0 + 1); box[3] = (int)(y1 - y0 + 1);
                }
            }
        }
    }
    // Moving bodies: the first step of a two-step launch takes a mask of its own, and so do the
    // first two of a three-step launch.
    if (moving && !s->mask_alt && hipMalloc(&s->mask_alt, (size_t)g.pitch * g.ny) != hipSuccess) {
        (void)hipGetLastError();
        s->mask_alt = nullptr;
        return fail(VPLBM_ENOMEM, "cannot allocate the second mask (%zu bytes)", (size_t)g.pitch * g.ny);
    }
    const bool third = moving && s->three_step && step3_supported(s->storage) &&
                       s->buf_bytes <= 0xFFFFFFFFu;
    if (third && !s->mask_alt2 && hipMalloc(&s->mask_alt2, (size_t)g.pitch * g.ny) != hipSuccess) {
        (void)hipGetLastError();
        s->mask_alt2 = nullptr;
        return fail(VPLBM_ENOMEM, "cannot allocate the third mask (%zu bytes)", (size_t)g.pitch * g.ny);
    }
    s->nbodies = nbodies;
    s->moving = moving;
    s->device_mask = body_id == nullptr;
    if (nbodies) HIP_TRY(hipMemcpyAsync(s->d_params, s->h_params, sizeof(BodyParams) * nbodies, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(launch_bodies(s->d_params, s->d_state, nbodies, s->t_dev, 0, s->stream));
    if (body_id) {
        HIP_TRY(hipMemcpy2DAsync(s->mask, g.pitch, body_id, g.nx, g.nx, g.ny, hipMemcpyHostToDevice, s->stream));
    } else {
        HIP_TRY(launch_mask(s->mask, g, s->d_params, s->d_state, nbodies, 0, 0, g.nx, g.ny, s->stream));
    }
    if (moving) {
        // The other masks: the whole lattice now; each launch of several steps then rebuilds
        // their swept boxes at the times of its first steps, and those of the simulation's own
        // at its last step's.
        HIP_TRY(launch_mask(s->mask_alt, g, s->d_params, s->d_state, nbodies, 0, 0, g.nx, g.ny, s->stream));
        if (s->mask_alt2)
            HIP_TRY(launch_mask(s->mask_alt2, g, s->d_params, s->d_state, nbodies, 0, 0, g.nx, g.ny, s->stream));
    }
    host_log("set_mask %p: %d bodies, moving %d, steps per launch %d", (void *)s, nbodies,
             moving ? 1 : 0, three_step_ok(s) ? 3 : two_step_ok(s) ? 2 : 1);
    if (s->steps == 0) {
        HIP_TRY(launch_init(s->storage, step_args(s, s->cur ^ 1, 0), nullptr, nullptr, nullptr, s->cfg.rho0, s->cfg.ux0, s->cfg.uy0, s->stream));
        HIP_TRY(reset_outlet(s));
    }
    HIP_TRY(hipStreamSynchronize(s->stream));   // body_id / bodies may be freed by the caller
    return VPLBM_OK;
}

int vplbm_step(vplbm_sim s, int64_t nsteps)
{
    if (!valid(s)) return fail(VPLBM_EINVAL, "invalid handle");
    if (nsteps < 0) return fail(VPLBM_EINVAL, "nsteps must be >= 0");
    if (s->unstable) return fail(VPLBM_EUNSTABLE, "the simulation became unstable (non-finite or non-positive density)");
    while (nsteps > 0) {
        const StepChunk c = next_chunk(nsteps, s->graph_k);
        if (c.graph) {
            int rc = ensure_graph(s, s->cur);
            if (rc) return rc;
            HIP_TRY(hipGraphLaunch(s->graph[s->cur], s->stream));
            s->cur ^= s->graph_flip[s->cur];
        } else {
            int flip = 0;
            HIP_TRY(enqueue_steps(s, s->cur, c.n, s->stream, &flip));
            s->cur ^= flip;
        }
        s->steps += c.n;
        nsteps -= c.n;
    }
    return VPLBM_OK;
}

int vplbm_observables(vplbm_sim s, vplbm_obs *out, double *rho, double *ux, double *uy)
{
    if (!valid(s)) return fail(VPLBM_EINVAL, "invalid handle");
    const Geom &g = s->g;
    const size_t n = (size_t)g.nx * g.ny;
    const bool fields = rho || ux || uy;
    double row[kRingWidth];
    unsigned status = 0;
    if (fields) {
        int rc = ensure_staging(s, 3 * n * sizeof(double));
        if (rc) return rc;
        if (s->moving) HIP_TRY(place_bodies(s, 0, s->stream));
        HIP_TRY(launch_readback(s->storage, step_args(s, s->cur, 0), s->staging, s->staging + n, s->staging + 2 * n, s->stream));
    }
    const int64_t last = s->steps - 1;
    if (last >= 0 && s->cfg.reduce) HIP_TRY(launch_fold(step_args(s, s->cur, 0), s->stream));
    if (last >= 0 && s->cfg.reduce)
        HIP_TRY(hipMemcpyAsync(row, s->ring + (size_t)(last % s->ring_len) * kRingWidth, sizeof row, hipMemcpyDeviceToHost, s->stream));
    else
        memset(row, 0, sizeof row);
    HIP_TRY(hipMemcpyAsync(&status, s->status, sizeof status, hipMemcpyDeviceToHost, s->stream));
    if (rho) HIP_TRY(hipMemcpyAsync(rho, s->staging, n * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    if (ux) HIP_TRY(hipMemcpyAsync(ux, s->staging + n, n * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    if (uy) HIP_TRY(hipMemcpyAsync(uy, s->staging + 2 * n, n * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (status & 1u) s->unstable = true;
    if (out) {
        memset(out, 0, sizeof *out);
        out->step = last;
        out->mass = row[0];
        for (int k = 0; k < kMaxBodies; k++) {
            out->fx[k] = row[1 + 2 * k];
            out->fy[k] = row[2 + 2 * k];
        }
        out->nbodies = s->nbodies;
        out->status = (status & 1u) ? 1 : 0;
    }
    return VPLBM_OK;
}

int vplbm_init_fields(vplbm_sim s, const double *rho, const double *ux, const double *uy)
{
    if (!valid(s)) return fail(VPLBM_EINVAL, "invalid handle");
    if (!rho || !ux || !uy) return fail(VPLBM_EINVAL, "rho, ux and uy are required");
    const size_t n = (size_t)s->g.nx * s->g.ny;
    int rc = ensure_staging(s, 3 * n * sizeof(double));
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(s->staging, rho, n * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->staging + n, ux, n * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->staging + 2 * n, uy, n * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(launch_init(s->storage, step_args(s, s->cur ^ 1, 0), s->staging, s->staging + n, s->staging + 2 * n, 0, 0, 0, s->stream));
    HIP_TRY(reset_outlet(s));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return VPLBM_OK;
}

int vplbm_get_populations(vplbm_sim s, double *pop)
{
    if (!valid(s) || !pop) return fail(VPLBM_EINVAL, "invalid handle or NULL output");
    const size_t n = (size_t)s->g.nx * s->g.ny;
    int rc = ensure_staging(s, 9 * n * sizeof(double));
    if (rc) return rc;
    HIP_TRY(launch_decode(s->storage, step_args(s, s->cur, 0), s->staging, s->stream));
    HIP_TRY(hipMemcpyAsync(pop, s->staging, 9 * n * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return VPLBM_OK;
}

int vplbm_set_populations(vplbm_sim s, const double *pop, int64_t step)
{
    if (!valid(s) || !pop) return fail(VPLBM_EINVAL, "invalid handle or NULL input");
    if (step < 0) return fail(VPLBM_EINVAL, "step must be >= 0");
    const size_t n = (size_t)s->g.nx * s->g.ny;
    int rc = ensure_staging(s, 9 * n * sizeof(double));
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(s->staging, pop, 9 * n * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(launch_encode(s->storage, step_args(s, s->cur ^ 1, 0), s->staging, s->stream));
    HIP_TRY(reset_outlet(s));
    long long t = step;
    HIP_TRY(hipMemcpyAsync(s->t_dev, &t, sizeof t, hipMemcpyHostToDevice, s->stream));
    HIP_TRY(launch_fill_f64(s->acc, (size_t)kAccSets * kSub * kRingWidth, 0.0, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->steps = step;
    return VPLBM_OK;
}

int vplbm_get_mask(vplbm_sim s, uint8_t *body_id)
{
    if (!valid(s) || !body_id) return fail(VPLBM_EINVAL, "invalid handle or NULL output");
    const Geom &g = s->g;
    HIP_TRY(hipMemcpy2DAsync(body_id, g.nx, s->mask, g.pitch, g.nx, g.ny, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    return VPLBM_OK;
}

int vplbm_force_series(vplbm_sim s, int64_t first, int64_t count, double *out)
{
    if (!valid(s) || (count > 0 && !out)) return fail(VPLBM_EINVAL, "invalid handle or NULL output");
    if (!s->cfg.reduce) return fail(VPLBM_ESTATE, "reductions are off (config.reduce = 0)");
    if (count < 0 || first < 0 || first + count > s->steps || first < s->steps - s->ring_len)
        return fail(VPLBM_EINVAL, "steps [%lld, %lld) are not in the ring (steps done %lld, ring %d)",
                    (long long)first, (long long)(first + count), (long long)s->steps, s->ring_len);
    if (s->steps >= 1) HIP_TRY(launch_fold(step_args(s, s->cur, 0), s->stream));
    int64_t done = 0;
    while (done < count) {
        const int64_t slot = (first + done) % s->ring_len;
        int64_t run = s->ring_len - slot;
        if (run > count - done) run = count - done;
        HIP_TRY(hipMemcpyAsync(out + done * kRingWidth, s->ring + slot * kRingWidth, run * kRingWidth * sizeof(double), hipMemcpyDeviceToHost, s->stream));
        done += run;
    }
    HIP_TRY(hipStreamSynchronize(s->stream));
    return VPLBM_OK;
}

int vplbm_momentum_exchange(vplbm_sim s, double *fx, double *fy)
{
    if (!valid(s) || !fx || !fy) return fail(VPLBM_EINVAL, "invalid handle or NULL output");
    int rc = ensure_staging(s, 2 * kMaxBodies * sizeof(double));
    if (rc) return rc;
    double out[2 * kMaxBodies];
    HIP_TRY(launch_fill_f64(s->staging, 2 * kMaxBodies, 0.0, s->stream));
    HIP_TRY(launch_momentum_exchange(s->storage, step_args(s, s->cur, 0), s->staging, s->stream));
    HIP_TRY(hipMemcpyAsync(out, s->staging, sizeof out, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    for (int k = 0; k < kMaxBodies; k++) {
        fx[k] = out[2 * k];
        fy[k] = out[2 * k + 1];
    }
    return VPLBM_OK;
}

int vplbm_momentum_exchange_noalloc(vplbm_sim s, double *out)
{
    if (!valid(s) || !out) return fail(VPLBM_EINVAL, "invalid handle or NULL output");
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, out) != hipSuccess ||
        (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)) {
        (void)hipGetLastError();
        return fail(VPLBM_EINVAL, "out must be device memory");
    }
    double *sp = static_scratch(s->device);
    if (!sp) return fail(VPLBM_EHIP, "the static scratch of device %d could not be located", s->device);
    return launch_exchange_static(s->storage, step_args(s, s->cur, 0), sp, out, s->stream);
}

int vplbm_residual(vplbm_sim s, double *residual)
{
    if (!valid(s) || !residual) return fail(VPLBM_EINVAL, "invalid handle or NULL output");
    const size_t n = (size_t)s->g.nx * s->g.ny;
    const int parts = residual_parts(s->g);
    if (!s->snap) {
        HIP_TRY(hipStreamSynchronize(s->stream));
        if (hipMalloc(&s->snap, 2 * n * sizeof(double)) != hipSuccess ||
            hipMalloc(&s->rpart, (2 * (size_t)parts + 2) * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            if (s->snap) (void)hipFree(s->snap);
            s->snap = nullptr;
            return fail(VPLBM_ENOMEM, "cannot allocate the residual snapshot (%zu bytes)", 2 * n * sizeof(double));
        }
        s->have_snap = false;
    }
    double sums[2];
    if (s->moving) HIP_TRY(place_bodies(s, 0, s->stream));   // the fields' time, as the readback
    HIP_TRY(launch_residual(s->storage, step_args(s, s->cur, 0), s->snap, s->rpart, s->rpart + 2 * parts, s->stream));
    HIP_TRY(hipMemcpyAsync(sums, s->rpart + 2 * parts, sizeof sums, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (!s->have_snap) *residual = INFINITY;
    else if (sums[1] > 0.0) *residual = sqrt(sums[0] / sums[1]);
    else *residual = sums[0] > 0.0 ? INFINITY : 0.0;
    s->have_snap = true;
    return VPLBM_OK;
}

int vplbm_steps_per_launch(vplbm_sim s, int32_t *steps)
{
    if (!valid(s) || !steps) return fail(VPLBM_EINVAL, "invalid handle or NULL output");
    *steps = three_step_ok(s) ? 3 : two_step_ok(s) ? 2 : 1;
    return VPLBM_OK;
}

int vplbm_steps_done(vplbm_sim s, int64_t *steps)
{
    if (!valid(s) || !steps) return fail(VPLBM_EINVAL, "invalid handle or NULL output");
    *steps = s->steps;
    return VPLBM_OK;
}

int vplbm_stream(vplbm_sim s, void **stream)
{
    if (!valid(s) || !stream) return fail(VPLBM_EINVAL, "invalid handle or NULL output");
    *stream = (void *)s->stream;
    return VPLBM_OK;
}

}  // extern "C"

// xf_api.hip -- the C ABI of libxf.so (declared in include/xf.h): argument
// checks on the host, then asynchronous launches on the caller's stream.
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>
#include <mutex>
#include <new>
#include <vector>

#include "xf_common.hpp"

namespace xf {
template <int N>
const NsOps *ops_ns();

const NsOps *ops_for_ns(int ns) {
    switch (ns) {
        case 1: return ops_ns<1>();
        case 2: return ops_ns<2>();
        case 3: return ops_ns<3>();
        case 4: return ops_ns<4>();
        case 5: return ops_ns<5>();
        case 6: return ops_ns<6>();
        case 7: return ops_ns<7>();
        case 8: return ops_ns<8>();
        case 9: return ops_ns<9>();
        default: return nullptr;
    }
}
}  // namespace xf

// Static device scratch of xf_rhs_noalloc: the workspace of a right-hand
// side for callers that cannot allocate.  Each device holds its own copy for
// the life of the process.  Host code never passes `scratch` itself (on the
// host it only names the symbol): it passes the device address resolved by
// hipGetSymbolAddress once per device (scratch_on_current_device).
constexpr size_t kScratchBytes = XF_NOALLOC_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of `scratch` on the current device (resolved on the first
// call per device), or nullptr when it cannot be resolved.
void *scratch_on_current_device(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

struct xf_ctx {
    xf::LaunchCtx lc;
    int ns, nv;
    const xf::NsOps *ops;
    int device;
    // per-kernel timing (off unless xf_timing enabled it)
    bool timing;
    int pp;   // positivity-preserving flux blend in the RK3 step
    int viscous;                // XF_VISCOUS_* bits, 0 = inviscid
    xf::TransportK *tk;         // device copy of the transport tables (xf_set_viscous)
    double W[XF_MAX_SPECIES];   // molar masses, kg/mol
    double a[XF_MAX_SPECIES][6];   // thermo coefficients a0..a5 of the table
    xf::ReactK *rk;             // device copy of the reaction mechanism (xf_set_reactions)
    int react_sub;              // alpha-QSS sub-steps per reaction step, 0 = no reactions
    int react_split;            // XF_SPLIT_STRANG or XF_SPLIT_LIE
    void *scratch;              // device address of the static scratch on this context's device
    struct Rec {
        int cls;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
};

namespace {

using xf::LaunchCtx;

constexpr size_t kAlign = 256;

size_t align_up(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

// Workspace carve-up (byte offsets); every piece 256-byte aligned.
struct Layout {
    size_t P, Pbar, mx, L, U0, S2, Ly, Lz, V0, V1, V2, lam0, mu, Uf, Pf, Q, G, Lf, Lv, total;
};

Layout layout(const xf_ctx *c, int op) {
    const size_t cell = (size_t)c->lc.g.cells * sizeof(double);
    const size_t state = cell * c->nv;
    Layout l{};
    size_t o = 0;
    l.P = o;
    o += align_up(4 * cell);
    l.mx = o;
    o += kAlign;
    if (c->lc.precision == XF_PREC_MIXED) {   // FP32 copies read by the mixed sweeps
        l.Uf = o;
        o += align_up((size_t)c->lc.g.cells * sizeof(float) * c->nv);
        l.Pf = o;
        o += align_up((size_t)c->lc.g.cells * sizeof(float) * 4);
    }
    if (c->viscous && (op == XF_OP_RHS || op == XF_OP_RK3)) {   // transport pass and velocity gradient
        l.Q = o;
        o += align_up(cell * xf::transport_fields(c->ns));
        l.G = o;
        o += align_up(cell * 9);
    }
    if (op == XF_OP_VJP || op == XF_OP_RK3_VJP) {
        l.Pbar = o;   // cotangents of each cell's p, T and rho
        o += align_up(3 * cell);
    }
    const bool mixed = c->lc.precision == XF_PREC_MIXED;
    if (mixed) {   // FP32 per-direction differences of the mixed sweeps, [3][Nv][cells]
        l.Lf = o;
        o += align_up((size_t)c->lc.g.cells * sizeof(float) * c->nv * 3);
    }
    if (op == XF_OP_RK3 && mixed && c->viscous) {   // FP64 viscous residual of a mixed step
        l.Lv = o;
        o += align_up(state);
    }
    if (op == XF_OP_RK3_VJP || (op == XF_OP_RK3 && !mixed)) {
        l.L = o;
        o += align_up(state);
    }
    if (op == XF_OP_RK3 || op == XF_OP_RK3_VJP) {
        l.U0 = o;
        o += align_up(state);
    }
    if (op == XF_OP_RK3) {
        l.S2 = o;
        o += align_up(state);
        if (!mixed) {
            l.Ly = o;
            o += align_up(state);
            l.Lz = o;
            o += align_up(state);
        }
    }
    if (op == XF_OP_RK3_VJP) {
        l.V0 = o;
        o += align_up(state);
        l.V1 = o;
        o += align_up(state);
        l.V2 = o;
        o += align_up(state);
        l.lam0 = l.U0;   // the forward stage buffer doubles as the adjoint accumulator
        l.mu = o;
        o += align_up(state);
    }
    l.total = o;
    return l;
}

template <typename T>
T *at(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

bool aligned8(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 7u) == 0; }

int dev_err(hipError_t e) { return e == hipSuccess ? XF_OK : XF_EDEVICE; }

#define XF_TRY(expr)                                  \
    do {                                              \
        const hipError_t _e = (expr);                 \
        if (_e != hipSuccess) return XF_EDEVICE;      \
    } while (0)

hipError_t take_event(xf_ctx *c, hipEvent_t *e) {
    if (!c->pool.empty()) {
        *e = c->pool.back();
        c->pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

// Run one launch (a callable returning hipError_t), bracketed by events
// when timing is on.
template <class F>
hipError_t timed(xf_ctx *c, int cls, hipStream_t s, F &&launch) {
    if (!c->timing) return launch();
    xf_ctx::Rec r{cls, nullptr, nullptr};
    hipError_t e = take_event(c, &r.a);
    if (e != hipSuccess) return e;
    if ((e = take_event(c, &r.b)) != hipSuccess) return e;
    if ((e = hipEventRecord(r.a, s)) != hipSuccess) return e;
    if ((e = launch()) != hipSuccess) return e;
    if ((e = hipEventRecord(r.b, s)) != hipSuccess) return e;
    c->recs.push_back(r);
    return hipSuccess;
}

// Primitive-variable buffers of one call: P (FP64), and for mixed-precision
// contexts the FP32 copies Uf, Pf that the sweeps read and the FP32
// per-direction differences they write.
struct Prim {
    double *P;
    float *Uf, *Pf;
    unsigned long long *mx;   // [0]: CFL maximum; [1 + 3 d .. 3 + 3 d]: GLF speeds of direction d
    double *Q, *G;            // transport pass and velocity gradient (viscous contexts)
    float *Lf;                // mixed: FP32 differences of direction d at Lf + d Nv cells
    long long lstride;        // Nv cells
    float *lf(int d) const { return Lf + d * lstride; }
};

Prim prim_bufs(const xf_ctx *c, const Layout &l, void *ws) {
    const bool mixed = c->lc.precision == XF_PREC_MIXED;
    const bool visc = c->viscous && l.G != 0;
    return {at<double>(ws, l.P),
            mixed ? at<float>(ws, l.Uf) : nullptr,
            mixed ? at<float>(ws, l.Pf) : nullptr,
            at<unsigned long long>(ws, l.mx),
            visc ? at<double>(ws, l.Q) : nullptr,
            visc ? at<double>(ws, l.G) : nullptr,
            mixed ? at<float>(ws, l.Lf) : nullptr,
            (long long)c->lc.g.cells * c->nv};
}

// Viscous fluxes of every active direction added to out[d] (the three may
// be one buffer): the transport pass and the velocity gradient, then one
// face kernel per direction.
int viscous_into(xf_ctx *c, const double *U, const Prim &pb, double *const out[3], hipStream_t s) {
    if (!c->viscous) return XF_OK;
    if (!pb.Q || !pb.G) return XF_EINVAL;
    const LaunchCtx &lc = c->lc;
    const int n[3] = {lc.g.nx, lc.g.ny, lc.g.nz};
    XF_TRY(timed(c, XF_K_TRANSPORT, s, [&] {
        hipError_t e = c->ops->transport(lc, U, pb.P, pb.Q, c->tk, s);
        if (e == hipSuccess) e = xf::launch_vel_grad(lc, pb.Q, pb.G, s);
        return e;
    }));
    for (int d = 0; d < 3; ++d) {
        if (n[d] <= 1) continue;
        XF_TRY(timed(c, XF_K_VISCOUS_X + d, s,
                     [&] { return c->ops->viscous(lc, d, U, pb.P, pb.Q, pb.G, out[d], c->viscous, s); }));
    }
    return XF_OK;
}

// GLF speeds of the active directions from the primitives just computed; a
// no-op for the other artificial viscosities.
hipError_t glf_speeds(xf_ctx *c, const double *U, const double *P, unsigned long long *mx, hipStream_t s) {
    if (c->lc.visc != XF_VISC_GLF) return hipSuccess;
    const int n[3] = {c->lc.g.nx, c->lc.g.ny, c->lc.g.nz};
    return timed(c, XF_K_CFL, s, [&] {
        hipError_t e = xf::launch_reset_u64(mx + 1, 9, s);
        for (int d = 0; d < 3 && e == hipSuccess; ++d)
            if (n[d] > 1) e = c->ops->glf(c->lc, d, U, P, mx + 1 + 3 * d, s);
        return e;
    });
}

const double *glf_of(const xf_ctx *c, const unsigned long long *mx, int d) {
    return c->lc.visc == XF_VISC_GLF ? reinterpret_cast<const double *>(mx + 1 + 3 * d) : nullptr;
}

// p64 = false: the FP64 primitives are not needed (the FP32 copies are).
// Ug = U: the pass also fills the ghosts of U it covers.  cfl: the pass also
// takes the CFL maximum into *cfl (zeroed beforehand)
hipError_t prims(xf_ctx *c, const double *U, const Prim &pb, hipStream_t s, bool p64 = true, double *Ug = nullptr,
                 unsigned long long *cfl = nullptr) {
    // viscous contexts: every padded cell (the tangential derivatives read edge ghosts)
    hipError_t e = timed(c, XF_K_PRIMS, s, [&] {
        return c->ops->prims(c->lc, U, p64 ? pb.P : nullptr, pb.Uf, pb.Pf, c->viscous ? 1 : 0, Ug, cfl, s);
    });
    if (e == hipSuccess) e = glf_speeds(c, U, pb.P, pb.mx, s);
    return e;
}

// The active sweeps into rhs, z, then y, then x.  FP64 contexts accumulate
// in rhs; mixed ones write one FP32 buffer per direction and sum them into
// rhs in FP64, in the same order.
int sweeps_into(xf_ctx *c, const double *U, double *rhs, const Prim &pb, hipStream_t s) {
    const LaunchCtx &lc = c->lc;
    const int n[3] = {lc.g.nx, lc.g.ny, lc.g.nz};
    const bool mixed = lc.precision == XF_PREC_MIXED;
    const xf::StageArgs off{};
    bool first = true;
    for (int d = 2; d >= 0; --d) {
        if (n[d] <= 1) continue;
        const int acc = first ? 0 : 1;
        XF_TRY(timed(c, XF_K_SWEEP_X + d, s, [&] {
            return c->ops->sweep(lc, d, mixed ? 0 : acc, U, pb.P, pb.Uf, pb.Pf, rhs, mixed ? pb.lf(d) : nullptr, off,
                                 glf_of(c, pb.mx, d), s);
        }));
        first = false;
    }
    if (first) return XF_EUNSUPPORTED;   // no active dimension (rejected by xf_create)
    if (mixed) {
        const float *const L[3] = {n[0] > 1 ? pb.lf(0) : nullptr, n[1] > 1 ? pb.lf(1) : nullptr,
                                   n[2] > 1 ? pb.lf(2) : nullptr};
        XF_TRY(timed(c, XF_K_STAGE, s, [&] { return xf::launch_sum_dirs(lc, c->nv, rhs, L, s); }));
    }
    return XF_OK;
}

int rhs_into(xf_ctx *c, const double *U, double *rhs, const Prim &pb, hipStream_t s) {
    XF_TRY(prims(c, U, pb, s));
    int r = sweeps_into(c, U, rhs, pb, s);
    if (r != XF_OK) return r;
    double *const all[3] = {rhs, rhs, rhs};
    if ((r = viscous_into(c, U, pb, all, s)) != XF_OK) return r;
    XF_TRY(timed(c, XF_K_ZERO, s, [&] { return xf::launch_zero_ghosts(c->lc, c->nv, rhs, s); }));
    return XF_OK;
}

int rhs_vjp_into(xf_ctx *c, const double *U, const double *rbar, double *Ubar, double *P, double *Pbar,
                 unsigned long long *mx, hipStream_t s) {
    const LaunchCtx &lc = c->lc;
    const int n[3] = {lc.g.nx, lc.g.ny, lc.g.nz};
    XF_TRY(timed(c, XF_K_PRIMS, s, [&] { return c->ops->prims(lc, U, P, nullptr, nullptr, 0, nullptr, nullptr, s); }));
    XF_TRY(glf_speeds(c, U, P, mx, s));
    XF_TRY(timed(c, XF_K_ZERO, s, [&] { return xf::launch_zero(3 * lc.g.cells, Pbar, s); }));
    for (int d = 0; d < 3; ++d) {
        if (n[d] <= 1) continue;
        XF_TRY(timed(c, XF_K_VJP_X + d, s,
                     [&] {
                         return c->ops->sweep_vjp(lc, d, U, P, rbar, Ubar, Pbar, glf_of(c, mx, d), s);
                     }));
    }
    XF_TRY(timed(c, XF_K_PRIMS_VJP, s, [&] { return c->ops->prims_vjp(lc, U, P, Pbar, Ubar, s); }));
    return XF_OK;
}

hipError_t fill(xf_ctx *c, double *U, hipStream_t s) {
    return timed(c, XF_K_FILL, s, [&] { return xf::launch_fill_ghosts(c->lc, c->nv, U, s); });
}

hipError_t fill_vjp(xf_ctx *c, double *Ub, hipStream_t s) {
    return timed(c, XF_K_FILL_VJP, s, [&] { return xf::launch_fill_ghosts_vjp(c->lc, c->nv, Ub, s); });
}

bool grid_ok(const xf_grid *g, int ng) {
    const int n[3] = {g->nx, g->ny, g->nz};
    const double d[3] = {g->dx, g->dy, g->dz};
    for (int k = 0; k < 3; ++k) {
        if (n[k] < 1 || n[k] > 65535) return false;
        if (n[k] > 1) {
            if (n[k] < ng) return false;
            if (!(d[k] > 0.0)) return false;
            const int a = g->bc[2 * k], b = g->bc[2 * k + 1];
            if ((a != XF_BC_PERIODIC && a != XF_BC_OUTFLOW) || (b != XF_BC_PERIODIC && b != XF_BC_OUTFLOW))
                return false;
            if ((a == XF_BC_PERIODIC) != (b == XF_BC_PERIODIC)) return false;
        }
    }
    if (n[0] <= 1 && n[1] <= 1 && n[2] <= 1) return false;
    const double cells = (double)(n[0] + (n[0] > 1 ? 2 * ng : 0)) * (n[1] + (n[1] > 1 ? 2 * ng : 0)) *
                         (n[2] + (n[2] > 1 ? 2 * ng : 0));
    return cells < 9.0e18 / 16.0;
}

template <typename R>
void fill_thermo(xf::ThermoK<R> &t, const xf_thermo *th) {
    memset(&t, 0, sizeof(t));
    for (int s = 0; s < th->ns; ++s) {
        const double Rs = xf::kRu / th->W[s];
        const double *a = th->a + 6 * s;
        t.Rs[s] = (R)Rs;
        t.cv[s][0] = (R)(Rs * (a[0] - 1.0));
        t.cv[s][1] = (R)(Rs * a[1]);
        t.cv[s][2] = (R)(Rs * a[2]);
        t.cv[s][3] = (R)(Rs * a[3]);
        t.cv[s][4] = (R)(Rs * a[4]);
        t.e[s][0] = (R)(Rs * a[5]);
        t.e[s][1] = (R)(Rs * (a[0] - 1.0));
        t.e[s][2] = (R)(Rs * a[1] / 2.0);
        t.e[s][3] = (R)(Rs * a[2] / 3.0);
        t.e[s][4] = (R)(Rs * a[3] / 4.0);
        t.e[s][5] = (R)(Rs * a[4] / 5.0);
    }
    t.bracket = th->T_hi > 0.0 ? 1 : 0;
    t.T_lo = th->T_lo;
    t.T_hi = th->T_hi;
    t.T_ref = t.bracket ? 0.5 * (th->T_lo + th->T_hi) : 1.0;
}

}  // namespace

extern "C" {

int xf_create(const xf_grid *grid, const xf_thermo *thermo, int precision, xf_ctx **out) {
    return xf_create_ghosts(grid, thermo, precision, 3, out);
}

int xf_create_ghosts(const xf_grid *grid, const xf_thermo *thermo, int precision, int ghost_width,
                     xf_ctx **out) {
    if (!out) return XF_EINVAL;
    *out = nullptr;
    if (ghost_width != 3 && ghost_width != 4) return XF_EINVAL;
    if (!grid || !thermo || !grid_ok(grid, ghost_width)) return XF_EINVAL;
    if (precision != XF_PREC_FP64 && precision != XF_PREC_MIXED) return XF_EINVAL;
    if (thermo->ns < 1 || !thermo->W || !thermo->a) return XF_EINVAL;
    if (thermo->ns > XF_MAX_SPECIES) return XF_EUNSUPPORTED;
    for (int s = 0; s < thermo->ns; ++s)
        if (!(thermo->W[s] > 0.0)) return XF_EINVAL;
    if (thermo->T_hi > 0.0 && !(thermo->T_lo < thermo->T_hi)) return XF_EINVAL;
    const xf::NsOps *ops = xf::ops_for_ns(thermo->ns);
    if (!ops) return XF_EUNSUPPORTED;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return XF_EDEVICE;
    xf_ctx *c = new (std::nothrow) xf_ctx();
    if (!c) return XF_ENOMEM;
    c->timing = false;
    c->pp = 0;
    c->viscous = 0;
    c->tk = nullptr;
    c->rk = nullptr;
    c->react_sub = 0;
    c->react_split = XF_SPLIT_STRANG;
    for (int s = 0; s < thermo->ns; ++s) {
        c->W[s] = thermo->W[s];
        for (int k = 0; k < 6; ++k) c->a[s][k] = thermo->a[s * 6 + k];
    }
    xf::Geo &g = c->lc.g;
    g.nx = grid->nx;
    g.ny = grid->ny;
    g.nz = grid->nz;
    g.gx = g.nx > 1 ? ghost_width : 0;
    g.gy = g.ny > 1 ? ghost_width : 0;
    g.gz = g.nz > 1 ? ghost_width : 0;
    g.px = g.nx + 2 * g.gx;
    g.py = g.ny + 2 * g.gy;
    g.pz = g.nz + 2 * g.gz;
    g.sy = g.px;
    g.sz = (long long)g.px * g.py;
    g.cells = g.sz * g.pz;
    g.dx = grid->dx;
    g.dy = grid->dy;
    g.dz = grid->dz;
    g.idx = g.nx > 1 ? 1.0 / grid->dx : 0.0;
    g.idy = g.ny > 1 ? 1.0 / grid->dy : 0.0;
    g.idz = g.nz > 1 ? 1.0 / grid->dz : 0.0;
    for (int k = 0; k < 6; ++k) g.bc[k] = grid->bc[k];
    fill_thermo(c->lc.th64, thermo);
    fill_thermo(c->lc.th32, thermo);
    c->lc.precision = precision;
    c->lc.visc = XF_VISC_LLF;
    c->lc.recon = XF_RECON_WENO5;
    c->ns = thermo->ns;
    c->nv = thermo->ns + 4;
    c->ops = ops;
    c->device = dev;
    c->scratch = scratch_on_current_device(dev);
    if (!c->scratch) {
        delete c;
        return XF_EDEVICE;
    }
    if (hipMalloc(reinterpret_cast<void **>(&c->lc.status), kAlign) != hipSuccess) {
        delete c;
        return XF_ENOMEM;
    }
    if (hipMemset(c->lc.status, 0, kAlign) != hipSuccess) {
        (void)hipFree(c->lc.status);
        delete c;
        return XF_EDEVICE;
    }
    *out = c;
    return XF_OK;
}

int xf_destroy(xf_ctx *c) {
    if (!c) return XF_EINVAL;
    for (auto &r : c->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : c->pool) (void)hipEventDestroy(e);
    if (c->tk) (void)hipFree(c->tk);
    if (c->rk) (void)hipFree(c->rk);
    const hipError_t e = hipFree(c->lc.status);
    delete c;
    return dev_err(e);
}

int xf_timing(xf_ctx *c, int enable) {
    if (!c) return XF_EINVAL;
    c->timing = enable != 0;
    return XF_OK;
}

int xf_timing_read(xf_ctx *c, void *stream, double *ms, long long *launches) {
    if (!c || !ms || !launches) return XF_EINVAL;
    XF_TRY(hipStreamSynchronize((hipStream_t)stream));
    for (int k = 0; k < XF_K_COUNT; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (auto &r : c->recs) {
        float t = 0.0f;
        XF_TRY(hipEventElapsedTime(&t, r.a, r.b));
        ms[r.cls] += t;
        launches[r.cls] += 1;
        c->pool.push_back(r.a);
        c->pool.push_back(r.b);
    }
    c->recs.clear();
    return XF_OK;
}

size_t xf_state_elems(const xf_ctx *c) { return c ? (size_t)c->lc.g.cells * c->nv : 0; }

size_t xf_workspace_bytes(const xf_ctx *c, int op) {
    if (!c || op < XF_OP_RHS || op > XF_OP_RK3_VJP) return 0;
    return layout(c, op).total;
}

int xf_fill_ghosts(xf_ctx *c, double *U, void *stream) {
    if (!c || !U || !aligned8(U)) return XF_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    return dev_err(fill(c, U, s));
}

int xf_fill_ghosts_vjp(xf_ctx *c, double *Ub, void *stream) {
    if (!c || !Ub || !aligned8(Ub)) return XF_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    return dev_err(fill_vjp(c, Ub, s));
}

int xf_rhs(xf_ctx *c, const double *U, double *rhs, void *ws, void *stream) {
    if (!c || !U || !rhs || !ws || U == rhs || !aligned8(U) || !aligned8(rhs) || !aligned8(ws))
        return XF_EINVAL;
    const Layout l = layout(c, XF_OP_RHS);
    return rhs_into(c, U, rhs, prim_bufs(c, l, ws), (hipStream_t)stream);
}

int xf_rhs_noalloc(xf_ctx *c, const double *U, double *rhs, void *stream) {
    if (!c || !U || !rhs || U == rhs || !aligned8(U) || !aligned8(rhs)) return XF_EINVAL;
    const Layout l = layout(c, XF_OP_RHS);
    if (l.total > kScratchBytes) return XF_ETOOLARGE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != c->device) return XF_EINVAL;
    // no event is created here: per-kernel timing skips this call's launches
    const bool timing = c->timing;
    c->timing = false;
    const int r = rhs_into(c, U, rhs, prim_bufs(c, l, c->scratch), (hipStream_t)stream);
    c->timing = timing;
    return r;
}

int xf_rhs_alpha(xf_ctx *c, const double *U, const double *alpha_in, double *alpha_out, double *rhs, void *ws,
                 void *stream) {
    if (!c || !U || !rhs || !ws || U == rhs || !aligned8(U) || !aligned8(rhs) || !aligned8(ws) ||
        !aligned8(alpha_in) || !aligned8(alpha_out))
        return XF_EINVAL;
    if (!alpha_in && !alpha_out) return xf_rhs(c, U, rhs, ws, stream);
    const Layout l = layout(c, XF_OP_RHS);
    const Prim pb = prim_bufs(c, l, ws);
    const hipStream_t s = (hipStream_t)stream;
    const LaunchCtx &lc = c->lc;
    XF_TRY(prims(c, U, pb, s));
    // per direction: [3][face count] speeds, directions in the order x, y, z
    long long off = 0;
    for (int d = 0; d < 3; ++d) {
        const long long nf = xf::face_count(lc.g, d);
        if (!nf) continue;
        if (alpha_out)
            XF_TRY(timed(c, XF_K_CFL, s, [&] {
                return c->ops->face_speeds(lc, d, U, pb.P, glf_of(c, pb.mx, d), alpha_out + off, nf, s);
            }));
        off += 3 * nf;
    }
    if (!alpha_in) {
        const int r = sweeps_into(c, U, rhs, pb, s);
        if (r != XF_OK) return r;
    } else {
        // every direction writes its own difference, then the sum goes to rhs
        // in the order z, y, x of the plain right-hand side
        off = 0;
        long long offs[3] = {0, 0, 0};
        for (int d = 0; d < 3; ++d) {
            offs[d] = off;
            off += 3 * xf::face_count(lc.g, d);
        }
        const bool mixed = lc.precision == XF_PREC_MIXED;
        bool first = true;
        for (int d = 2; d >= 0; --d) {
            const long long nf = xf::face_count(lc.g, d);
            if (!nf) continue;
            XF_TRY(timed(c, XF_K_SWEEP_X + d, s, [&] {
                return c->ops->sweep_frozen(lc, d, (first || mixed) ? 0 : 1, U, pb.P, pb.Uf, pb.Pf, rhs,
                                            mixed ? pb.lf(d) : nullptr, alpha_in + offs[d], nf, s);
            }));
            first = false;
        }
        if (mixed) {
            const float *const L[3] = {xf::face_count(lc.g, 0) ? pb.lf(0) : nullptr,
                                       xf::face_count(lc.g, 1) ? pb.lf(1) : nullptr,
                                       xf::face_count(lc.g, 2) ? pb.lf(2) : nullptr};
            XF_TRY(timed(c, XF_K_STAGE, s, [&] { return xf::launch_sum_dirs(lc, c->nv, rhs, L, s); }));
        }
    }
    double *const all[3] = {rhs, rhs, rhs};
    const int r = viscous_into(c, U, pb, all, s);
    if (r != XF_OK) return r;
    XF_TRY(timed(c, XF_K_ZERO, s, [&] { return xf::launch_zero_ghosts(c->lc, c->nv, rhs, s); }));
    return XF_OK;
}

int xf_primitives(xf_ctx *c, const double *U, double *prim, void *stream) {
    if (!c || !U || !prim || !aligned8(U) || !aligned8(prim)) return XF_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    XF_TRY(timed(c, XF_K_PRIMS, s, [&] { return c->ops->prims(c->lc, U, prim, nullptr, nullptr, 1, nullptr, nullptr, s); }));
    return XF_OK;
}

int xf_cfl_dt(xf_ctx *c, const double *U, double cfl, double *dt_dev, void *ws, void *stream) {
    if (!c || !U || !dt_dev || !ws || !(cfl > 0.0) || !aligned8(U) || !aligned8(ws)) return XF_EINVAL;
    const Layout l = layout(c, XF_OP_RHS);
    const hipStream_t s = (hipStream_t)stream;
    double *P = at<double>(ws, l.P);
    unsigned long long *mx = at<unsigned long long>(ws, l.mx);
    XF_TRY(timed(c, XF_K_PRIMS, s, [&] { return c->ops->prims(c->lc, U, P, nullptr, nullptr, 0, nullptr, nullptr, s); }));
    XF_TRY(timed(c, XF_K_CFL, s, [&] {
        hipError_t e = xf::launch_cfl_reset(mx, s);
        if (e == hipSuccess) e = c->ops->cfl(c->lc, U, P, mx, s);
        if (e == hipSuccess) e = xf::launch_cfl_finish(mx, cfl, dt_dev, s);
        return e;
    }));
    return XF_OK;
}

// One SSP-RK3 step.  Every sweep writes its own residual buffer (stores
// only: no read-modify-write inside the register-heavy sweep kernels; FP32
// buffers in mixed contexts, whose sweeps compute the differences in FP32),
// and a light stage kernel sums them in FP64 and applies the stage
// combination (ping-pong stage buffers S1, S2; stage 3 writes U in place).  With cfl > 0 the time
// step is reduced on the device from the stage-1 primitives of U^n and
// written to *dt_out before it is used.
int flow_rk3_step(xf_ctx *c, double *U, double dt, const double *dt_in, double cfl, double *dt_out, void *ws,
                  hipStream_t s);

// One reaction step over scale * dt (or *dt_dev), then the ghost fill.
int react_into(xf_ctx *c, double *U, double dt, const double *dt_dev, double scale, hipStream_t s) {
    XF_TRY(timed(c, XF_K_REACT, s,
                 [&] { return c->ops->react(c->lc, U, c->rk, dt, dt_dev, scale, c->react_sub, s); }));
    return fill(c, U, s) == hipSuccess ? XF_OK : XF_EDEVICE;
}

// The step of the context: the flow step alone, or split with the
// reaction step (Strang R(dt/2) F(dt) R(dt/2), or Lie-Trotter F(dt) R(dt)).
// With cfl > 0 and reactions, dt comes from U^n before the first reaction
// step and the flow step then uses it.
int rk3_step(xf_ctx *c, double *U, double dt, const double *dt_in, double cfl, double *dt_out, void *ws,
             hipStream_t s) {
    if (!c->react_sub) return flow_rk3_step(c, U, dt, dt_in, cfl, dt_out, ws, s);
    const double *h = dt_in;
    if (cfl > 0.0) {
        const Layout l = layout(c, XF_OP_RK3);
        const Prim pb = prim_bufs(c, l, ws);
        XF_TRY(fill(c, U, s));
        XF_TRY(prims(c, U, pb, s));
        XF_TRY(timed(c, XF_K_CFL, s, [&] {
            hipError_t e = xf::launch_cfl_reset(pb.mx, s);
            if (e == hipSuccess) e = c->ops->cfl(c->lc, U, pb.P, pb.mx, s);
            if (e == hipSuccess) e = xf::launch_cfl_finish(pb.mx, cfl, dt_out, s);
            return e;
        }));
        h = dt_out;
    }
    int r;
    if (c->react_split == XF_SPLIT_STRANG) {
        if ((r = react_into(c, U, dt, h, 0.5, s)) != XF_OK) return r;
    }
    if ((r = flow_rk3_step(c, U, dt, h, 0.0, nullptr, ws, s)) != XF_OK) return r;
    return react_into(c, U, dt, h, c->react_split == XF_SPLIT_STRANG ? 0.5 : 1.0, s);
}

int flow_rk3_step(xf_ctx *c, double *U, double dt, const double *dt_in, double cfl, double *dt_out, void *ws,
                  hipStream_t s) {
    const Layout l = layout(c, XF_OP_RK3);
    const LaunchCtx &lc = c->lc;
    const int n[3] = {lc.g.nx, lc.g.ny, lc.g.nz};
    const bool mixed = lc.precision == XF_PREC_MIXED;
    const Prim pb = prim_bufs(c, l, ws);
    double *P = pb.P;
    double *S1 = at<double>(ws, l.U0), *S2 = at<double>(ws, l.S2);
    // per-direction residuals: FP64 buffers, or the FP32 ones of a mixed context
    double *Ld[3] = {nullptr, nullptr, nullptr};
    if (!mixed) {
        Ld[0] = at<double>(ws, l.L);
        Ld[1] = at<double>(ws, l.Ly);
        Ld[2] = at<double>(ws, l.Lz);
    }
    const double *L64[3] = {nullptr, nullptr, nullptr};
    const float *L32[3] = {nullptr, nullptr, nullptr};
    for (int d = 0; d < 3; ++d) {
        if (n[d] <= 1) continue;
        if (mixed)
            L32[d] = pb.lf(d);
        else
            L64[d] = Ld[d];
    }
    // the viscous residual: into each direction's FP64 buffer, or into one
    // FP64 buffer of its own in a mixed context
    double *Lv = mixed && c->viscous ? at<double>(ws, l.Lv) : nullptr;
    double *const vout[3] = {Lv ? Lv : Ld[0], Lv ? Lv : Ld[1], Lv ? Lv : Ld[2]};
    const long long nstate = lc.g.cells * c->nv;
    unsigned long long *mx = at<unsigned long long>(ws, l.mx);
    const double *h = dt_in;
    double *in[3] = {U, S1, S2};
    double *out[3] = {S1, S2, U};
    const double a[3] = {0.0, 0.75, 1.0 / 3.0};
    const double b[3] = {1.0, 0.25, 2.0 / 3.0};
    // a mixed step without viscous terms or GLF needs only the FP32 copies
    // (the CFL maximum comes from the primitive pass itself)
    const bool p64 = !mixed || c->viscous || lc.visc == XF_VISC_GLF;
    // the primitive pass fills the ghosts of the stage input itself: the
    // face ghosts, and with viscous terms (whose tangential derivatives read
    // them) the edge and corner ghosts too; the state's ghosts are filled in
    // full at the end of the step
    // the CFL maximum of U^n (Eq. 17) is taken by the first primitive pass
    for (int k = 0; k < 3; ++k) {
        const bool take_cfl = k == 0 && cfl > 0.0;
        if (take_cfl) XF_TRY(timed(c, XF_K_CFL, s, [&] { return xf::launch_cfl_reset(mx, s); }));
        XF_TRY(prims(c, in[k], pb, s, p64, in[k], take_cfl ? mx : nullptr));
        if (take_cfl) {
            XF_TRY(timed(c, XF_K_CFL, s, [&] { return xf::launch_cfl_finish(mx, cfl, dt_out, s); }));
            h = dt_out;
        }
        // the step size for the positivity blend.  In a mixed context without
        // viscous terms or the blend the x sweep, which runs last, also
        // finishes the stage (Eq. 16): measured at 256^3, nine species, the
        // mixed step gains 0.4 ms, while the FP64 x sweep, at three waves per
        // SIMD, loses more than the separate stage kernel costs (4.05 against
        // 2.06 + 1.87 ms), so FP64 keeps that kernel
        xf::StageArgs sw{dt, h, c->pp};
        const bool fuse = mixed && !c->viscous && !c->pp && n[0] > 1;
        if (fuse) {
            sw.Uout = out[k];
            sw.U0 = U;
            sw.Uin = in[k];
            sw.Ly64 = L64[1];
            sw.Lz64 = L64[2];
            sw.Ly32 = L32[1];
            sw.Lz32 = L32[2];
            sw.a = a[k];
            sw.b = b[k];
        }
        for (int d = 2; d >= 0; --d) {
            if (n[d] <= 1) continue;
            XF_TRY(timed(c, XF_K_SWEEP_X + d, s, [&] {
                return c->ops->sweep(lc, d, 0, in[k], P, pb.Uf, pb.Pf, Ld[d], mixed ? pb.lf(d) : nullptr, sw,
                                     glf_of(c, pb.mx, d), s);
            }));
        }
        if (fuse) continue;
        if (Lv) XF_TRY(timed(c, XF_K_ZERO, s, [&] { return xf::launch_zero(nstate, Lv, s); }));
        const int r = viscous_into(c, in[k], pb, vout, s);
        if (r != XF_OK) return r;
        XF_TRY(timed(c, XF_K_STAGE, s, [&] {
            return c->ops->stage(lc, out[k], U, in[k], L64, L32, Lv, a[k], b[k], dt, h, s);
        }));
    }
    XF_TRY(fill(c, U, s));
    return XF_OK;
}

int xf_set_dissipation(xf_ctx *c, int type) {
    if (!c) return XF_EINVAL;
    if (type != XF_VISC_LLF && type != XF_VISC_ROE && type != XF_VISC_GLF) return XF_EINVAL;
    c->lc.visc = type;
    return XF_OK;
}

int xf_set_reconstruction(xf_ctx *c, int type) {
    if (!c) return XF_EINVAL;
    if (type != XF_RECON_WENO5 && type != XF_RECON_CU6 && type != XF_RECON_WENO7) return XF_EINVAL;
    const xf::Geo &g = c->lc.g;
    if (type == XF_RECON_WENO7 && (g.gx > 0 ? g.gx : g.gy > 0 ? g.gy : g.gz) < 4) return XF_EUNSUPPORTED;
    c->lc.recon = type;
    return XF_OK;
}

int xf_set_viscous(xf_ctx *c, const xf_transport *tr, int terms) {
    if (!c) return XF_EINVAL;
    if (terms & ~(XF_VISCOUS_STRESS | XF_VISCOUS_HEAT | XF_VISCOUS_DIFFUSION)) return XF_EINVAL;
    if (terms == 0) {
        c->viscous = 0;
        return XF_OK;
    }
    const int ns = c->ns;
    if (!tr || tr->ns != ns || !tr->mu || !tr->kappa || !tr->D || !(tr->p_ref > 0.0) || !std::isfinite(tr->p_ref))
        return XF_EINVAL;
    xf::TransportK h;
    memset(&h, 0, sizeof(h));
    for (int s = 0; s < ns; ++s) {
        for (int k = 0; k < 4; ++k) {
            h.mu[s][k] = tr->mu[s * 4 + k];
            h.kappa[s][k] = tr->kappa[s * 4 + k];
            if (!std::isfinite(h.mu[s][k]) || !std::isfinite(h.kappa[s][k])) return XF_EINVAL;
        }
        for (int t = 0; t < ns; ++t)
            for (int k = 0; k < 4; ++k) {
                const double v = tr->D[(s * ns + t) * 4 + k];
                if (!std::isfinite(v) || v != tr->D[(t * ns + s) * 4 + k]) return XF_EINVAL;
                h.D[s][t][k] = v;
            }
        h.W[s] = c->W[s];
        h.iW[s] = 1.0 / c->W[s];
    }
    for (int s = 0; s < ns; ++s)
        for (int t = 0; t < ns; ++t) {
            h.wa[s][t] = 1.0 / (std::sqrt(8.0) * std::sqrt(1.0 + c->W[s] / c->W[t]));
            h.wb[s][t] = std::pow(c->W[t] / c->W[s], 0.25);
        }
    h.ip_ref = 1.0 / tr->p_ref;
    if (!c->tk && hipMalloc(reinterpret_cast<void **>(&c->tk), sizeof(xf::TransportK)) != hipSuccess) {
        c->tk = nullptr;
        return XF_ENOMEM;
    }
    if (hipMemcpy(c->tk, &h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess) return XF_EDEVICE;
    c->viscous = terms;
    return XF_OK;
}

int xf_set_reactions(xf_ctx *c, const xf_mechanism *m, int substeps, int splitting) {
    if (!c) return XF_EINVAL;
    if (!m || substeps == 0) {
        c->react_sub = 0;
        return XF_OK;
    }
    const int ns = c->ns;
    if (substeps < 0 || (splitting != XF_SPLIT_STRANG && splitting != XF_SPLIT_LIE)) return XF_EINVAL;
    if (m->ns != ns || m->nr < 1 || m->nr > XF_MAX_REACTIONS || !m->nu_f || !m->nu_b || !m->A || !m->B || !m->E ||
        !m->third || !m->eff || !m->reversible || !m->s0)
        return XF_EINVAL;
    xf::ReactK h;
    memset(&h, 0, sizeof(h));
    h.nr = m->nr;
    double wmax = 0.0;
    for (int s = 0; s < ns; ++s) wmax = c->W[s] > wmax ? c->W[s] : wmax;
    for (int r = 0; r < m->nr; ++r) {
        if (!(m->A[r] > 0.0) || !std::isfinite(m->A[r]) || !std::isfinite(m->B[r]) || !std::isfinite(m->E[r]))
            return XF_EINVAL;
        if ((m->third[r] != 0 && m->third[r] != 1) || (m->reversible[r] != 0 && m->reversible[r] != 1))
            return XF_EINVAL;
        double dm = 0.0;
        int dn = 0;
        for (int s = 0; s < ns; ++s) {
            const int f = m->nu_f[r * ns + s], b = m->nu_b[r * ns + s];
            if (f < 0 || f > 3 || b < 0 || b > 3) return XF_EINVAL;
            const double e = m->eff[r * ns + s];
            if (!std::isfinite(e) || e < 0.0) return XF_EINVAL;
            h.nf[r][s] = f;
            h.nb[r][s] = b;
            h.fd[r][s] = f;
            h.bd[r][s] = b;
            for (int k = 0; k < f; ++k) {
                const unsigned n = h.fl[r] & 7u;
                if (n == 7u) return XF_EINVAL;   // more than seven reactant molecules
                h.fl[r] = (h.fl[r] + 1u) | ((unsigned)s << (3 + 4 * n));
            }
            for (int k = 0; k < b; ++k) {
                const unsigned n = h.bl[r] & 7u;
                if (n == 7u) return XF_EINVAL;   // more than seven product molecules
                h.bl[r] = (h.bl[r] + 1u) | ((unsigned)s << (3 + 4 * n));
            }
            h.eff[r][s] = e;
            dn += b - f;
            dm += c->W[s] * (b - f);
        }
        if (std::fabs(dm) > 1e-9 * wmax) return XF_EINVAL;   // the reaction must conserve mass
        h.dn[r] = dn;
        h.third[r] = m->third[r];
        h.rev[r] = m->reversible[r];
        h.lnA[r] = std::log(m->A[r]);
        h.B[r] = m->B[r];
        h.ER[r] = m->E[r] / xf::kRu;
    }
    h.th = c->lc.th64;
    h.lp0 = std::log(xf::kP0 / xf::kRu);
    for (int s = 0; s < ns; ++s) {
        if (!std::isfinite(m->s0[s])) return XF_EINVAL;
        h.W[s] = c->W[s];
        h.iW[s] = 1.0 / c->W[s];
    }
    // g_s = S/R - h/(R T) = a0 (ln T - 1) + a1 T/2 + a2 T^2/6 + a3 T^3/12
    //       + a4 T^4/20 - a5/T + a6, summed with the net coefficients
    static const double kGibbs[7] = {1.0, 1.0 / 2.0, 1.0 / 6.0, 1.0 / 12.0, 1.0 / 20.0, -1.0, 1.0};
    for (int r = 0; r < m->nr; ++r)
        for (int k = 0; k < 7; ++k) {
            double acc = 0.0;
            for (int s = 0; s < ns; ++s) {
                const int nu = h.nb[r][s] - h.nf[r][s];
                if (nu) acc += nu * (k < 6 ? c->a[s][k] : m->s0[s]);
            }
            h.G[r][k] = acc * kGibbs[k];
        }
    if (!c->rk && hipMalloc(reinterpret_cast<void **>(&c->rk), sizeof(xf::ReactK)) != hipSuccess) {
        c->rk = nullptr;
        return XF_ENOMEM;
    }
    if (hipMemcpy(c->rk, &h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess) return XF_EDEVICE;
    c->react_sub = substeps;
    c->react_split = splitting;
    return XF_OK;
}

int xf_react(xf_ctx *c, double *U, double dt, const double *dt_dev, void *stream) {
    if (!c || !U || !aligned8(U) || !(dt >= 0.0)) return XF_EINVAL;
    if (!c->react_sub) return XF_EUNSUPPORTED;
    return react_into(c, U, dt, dt_dev, 1.0, (hipStream_t)stream);
}

int xf_set_positivity(xf_ctx *c, int enable) {
    if (!c) return XF_EINVAL;
    c->pp = enable != 0;
    return XF_OK;
}

int xf_rk3_step(xf_ctx *c, double *U, double dt, const double *dt_dev, void *ws, void *stream) {
    if (!c || !U || !ws || !aligned8(U) || !aligned8(ws)) return XF_EINVAL;
    if (!dt_dev && !(dt >= 0.0)) return XF_EINVAL;
    return rk3_step(c, U, dt, dt_dev, 0.0, nullptr, ws, (hipStream_t)stream);
}

int xf_rk3_step_cfl(xf_ctx *c, double *U, double cfl, double *dt_dev, void *ws, void *stream) {
    if (!c || !U || !ws || !dt_dev || !(cfl > 0.0) || !aligned8(U) || !aligned8(ws) || !aligned8(dt_dev))
        return XF_EINVAL;
    return rk3_step(c, U, 0.0, nullptr, cfl, dt_dev, ws, (hipStream_t)stream);
}

int xf_rhs_vjp(xf_ctx *c, const double *U, const double *rbar, double *Ubar, void *ws, void *stream) {
    if (!c || !U || !rbar || !Ubar || !ws || Ubar == U || Ubar == rbar || !aligned8(U) || !aligned8(rbar) ||
        !aligned8(Ubar) || !aligned8(ws))
        return XF_EINVAL;
    if (c->lc.recon == XF_RECON_WENO7 || c->viscous || c->react_sub) return XF_EUNSUPPORTED;
    const Layout l = layout(c, XF_OP_VJP);
    return rhs_vjp_into(c, U, rbar, Ubar, at<double>(ws, l.P), at<double>(ws, l.Pbar),
                        at<unsigned long long>(ws, l.mx), (hipStream_t)stream);
}

int xf_rk3_step_vjp(xf_ctx *c, const double *Un, double dt, double *Ubar, void *ws, void *stream) {
    if (!c || !Un || !Ubar || !ws || Un == Ubar || !aligned8(Un) || !aligned8(Ubar) || !aligned8(ws) ||
        !(dt >= 0.0))
        return XF_EINVAL;
    if (c->pp) return XF_EUNSUPPORTED;   // the adjoint is of the unblended step
    if (c->lc.recon == XF_RECON_WENO7 || c->viscous || c->react_sub) return XF_EUNSUPPORTED;
    const Layout l = layout(c, XF_OP_RK3_VJP);
    const hipStream_t s = (hipStream_t)stream;
    const LaunchCtx &lc = c->lc;
    const long long n = lc.g.cells * c->nv;
    const Prim pb = prim_bufs(c, l, ws);
    double *P = pb.P, *Pbar = at<double>(ws, l.Pbar), *L = at<double>(ws, l.L);
    double *V0 = at<double>(ws, l.V0), *V1 = at<double>(ws, l.V1), *V2 = at<double>(ws, l.V2);
    double *lam0 = at<double>(ws, l.lam0), *mu = at<double>(ws, l.mu);
    int r;
    // forward stage states V0 = G(U_n), V1 = G(V0 + dt L(V0)), V2 = G(3/4 V0 + 1/4 (V1 + dt L(V1)))
    XF_TRY(timed(c, XF_K_STAGE, s, [&] { return xf::launch_copy(n, Un, V0, s); }));
    XF_TRY(fill(c, V0, s));
    if ((r = rhs_into(c, V0, L, pb, s)) != XF_OK) return r;
    XF_TRY(timed(c, XF_K_STAGE, s, [&] {
        hipError_t e = xf::launch_copy(n, V0, V1, s);
        if (e == hipSuccess) e = xf::launch_axpy_state(n, dt, L, 1.0, V1, s);
        return e;
    }));
    XF_TRY(fill(c, V1, s));
    if ((r = rhs_into(c, V1, L, pb, s)) != XF_OK) return r;
    XF_TRY(timed(c, XF_K_STAGE, s, [&] {
        hipError_t e = xf::launch_copy(n, V1, V2, s);
        if (e == hipSuccess) e = xf::launch_axpy_state(n, dt, L, 1.0, V2, s);
        if (e == hipSuccess) e = xf::launch_axpy_state(n, 0.75, V0, 0.25, V2, s);
        return e;
    }));
    XF_TRY(fill(c, V2, s));
    // reverse sweep through the stages
    double *const Vs[3] = {V0, V1, V2};
    XF_TRY(fill_vjp(c, Ubar, s));
    for (int stage = 3; stage >= 1; --stage) {
        XF_TRY(timed(c, XF_K_ZERO, s, [&] { return xf::launch_zero(n, mu, s); }));
        if ((r = rhs_vjp_into(c, Vs[stage - 1], Ubar, mu, P, Pbar, at<unsigned long long>(ws, l.mx), s)) != XF_OK)
            return r;
        XF_TRY(timed(c, XF_K_STAGE, s,
                     [&] { return xf::launch_rk3_stage_vjp(lc, c->nv, stage, Ubar, lam0, mu, nullptr, dt, s); }));
        if (stage > 1) XF_TRY(fill_vjp(c, Ubar, s));
    }
    XF_TRY(fill_vjp(c, lam0, s));
    XF_TRY(timed(c, XF_K_STAGE, s, [&] { return xf::launch_copy(n, lam0, Ubar, s); }));
    return XF_OK;
}

int xf_status(xf_ctx *c, void *stream, unsigned *flags_out) {
    if (!c || !flags_out) return XF_EINVAL;
    const hipStream_t s = (hipStream_t)stream;
    unsigned h = 0;
    const unsigned zero = 0;
    XF_TRY(hipMemcpyAsync(&h, c->lc.status, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    XF_TRY(hipMemcpyAsync(c->lc.status, &zero, sizeof(unsigned), hipMemcpyHostToDevice, s));
    XF_TRY(hipStreamSynchronize(s));
    *flags_out = h;
    return h ? XF_ENONPHYS : XF_OK;
}

const char *xf_strerror(int code) {
    switch (code) {
        case XF_OK: return "success";
        case XF_EINVAL: return "invalid argument";
        case XF_EDEVICE: return "HIP runtime error";
        case XF_ENOMEM: return "device allocation failed";
        case XF_ENONPHYS: return "non-physical state flagged by the kernels";
        case XF_EUNSUPPORTED: return "unsupported request (species count or operation)";
        case XF_ETOOLARGE: return "problem too large for the library's static scratch buffer";
        default: return "unknown status code";
    }
}

}  // extern "C"

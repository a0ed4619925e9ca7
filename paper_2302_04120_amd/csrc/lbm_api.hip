// C-ABI layer of liblbm: argument checks, the SI parameter compiler, the
// layout of the caller-owned device buffer, and the enqueue loops.  No device
// memory is allocated here; every kernel runs on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "lbm_internal.h"

using namespace lbm;

namespace {

// ---- scratch of lbm_reduce_noalloc -------------------------------------------
// The reduction partials (batch x 4 fields x kRedBlocks FP64) and the per-
// replica results (batch x 4) of that entry point live in this file-scope
// device array instead of the caller's buffer, for at most kNoAllocMaxBatch
// replicas (8.4 MB held on every GPU the library runs on until the process
// ends).  The host name `scratch` is only a stand-in for the symbol: host code
// uses the per-device address from hipGetSymbolAddress, taken once per device
// by the first lbm_create on it.  Every element the reduction reads is written
// earlier in the same call (each first-pass block writes its partials, the
// second pass every result), so nothing needs clearing between calls; calls
// that overlap on one GPU share the array and race.
constexpr int kNoAllocMaxBatch = 1024;
constexpr size_t kNoAllocDoubles = (size_t)kNoAllocMaxBatch * (4 * kRedBlocks + 4);
__device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device` (the current device), taken on
// the first call for that device; nullptr if the query fails.
double* scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[device] = static_cast<double*>(p);
    }
    return g_scratch_ptr[device];
}

constexpr uint32_t kMagic = 0x534d424cu;  // "LBMS"
constexpr uint32_t kVersion = 4;

struct Layout {
    long long N = 0, P = 0;
    int npop = 0, nplanes = 0;
    size_t es = 0;
    size_t offA = 0, offB = 0, offAux = 0, offStage = 0, offPartial = 0, offPhi = 0;
    size_t offSmall = 0, offFlags = 0, offWatch = 0, total = 0;
};

// Extra elements per value array (a multiple of 64).  P = N rounded up to 64
// plus this pad sizes each state buffer (nplanes P values, the node blocks at
// its start) and spaces the planes of the FP64 staging fields and of the 1D
// lattices.  When the states were stored as planes, planes a power of two
// apart (a 256^3 box, a batch of 2^k 256^2 cells) started at addresses
// congruent modulo every power of two up to the plane size, so the 19-38
// streams of a step hit the same HBM channels at once, and this spacing
// spread them (256^3 D3Q19 step: 27.8 -> 31.0 GLUPS; 67 M-node single-step
// phase kernel: 2.45 -> 2.25 ms).
#ifndef LBM_PLANE_PAD
#define LBM_PLANE_PAD 16448
#endif

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

lbm_status check_desc(const lbm_desc* d, Layout* L, std::string* err) {
    auto fail = [&](lbm_status st, const char* m) {
        if (err) *err = m;
        return st;
    };
    if (!d) return fail(LBM_E_ARG, "desc is NULL");
    if (d->nx < 1 || d->ny < 1 || d->batch < 1) return fail(LBM_E_ARG, "nx, ny, batch must be >= 1");
    if (d->prec != LBM_FP32_DEV && d->prec != LBM_FP64 && d->prec != LBM_FP32_DEV_ARITH64)
        return fail(LBM_E_ARG, "unknown precision");
    if (d->prec == LBM_FP32_DEV_ARITH64 && d->lattice != LBM_D2Q9_PHASE)
        return fail(LBM_E_UNSUPPORTED, "FP64 arithmetic on FP32 storage: LBM_D2Q9_PHASE only");
    if (d->batch > 65535 || d->ny > 65535 * 4) return fail(LBM_E_ARG, "grid too large for the launch geometry");
    for (int s = 0; s < 4; ++s)
        if (d->bc[s] < LBM_BC_PERIODIC || d->bc[s] > LBM_BC_SYMMETRY) return fail(LBM_E_ARG, "unknown boundary kind");
    const bool d3 = d->lattice == LBM_D3Q19 || d->lattice == LBM_D3Q19_PHASE;
    if (d3 ? d->nz < 1 : (d->nz < 0 || d->nz > 1 || d->bc_z[0] != 0 || d->bc_z[1] != 0))
        return fail(LBM_E_ARG, d3 ? "nz must be >= 1" : "nz and bc_z are for LBM_D3Q19 (0 or 1, and 0)");
    const long long nz = d3 ? d->nz : 1;
    Layout l;
    l.N = (long long)d->batch * d->nx * d->ny * nz;
    l.P = (l.N + 63) / 64 * 64 + LBM_PLANE_PAD;
    l.es = d->prec == LBM_FP64 ? 8 : 4;
    switch (d->lattice) {
        case LBM_D1Q2:
        case LBM_D1Q3:
            if (d->prec != LBM_FP64) return fail(LBM_E_UNSUPPORTED, "1D lattices run in FP64 only");
            if (d->ny != 1 || d->batch != 1) return fail(LBM_E_ARG, "1D lattices need ny = batch = 1");
            if (d->nx < 3 || d->nx > 1024) return fail(LBM_E_UNSUPPORTED, "1D lattices need 3 <= nx <= 1024");
            if (d->bc[0] != LBM_BC_DIRICHLET || d->bc[1] != LBM_BC_DIRICHLET)
                return fail(LBM_E_UNSUPPORTED, "1D lattices need Dirichlet ends");
            l.npop = d->lattice == LBM_D1Q2 ? 2 : 3;
            l.P = d->nx;
            break;
        case LBM_D2Q9_D2Q5: {
            const bool xp = d->bc[0] == LBM_BC_PERIODIC && d->bc[1] == LBM_BC_PERIODIC;
            const bool xio = d->bc[0] == LBM_BC_VEL_INLET && d->bc[1] == LBM_BC_P_OUTLET;
            const bool xd = d->bc[0] == LBM_BC_DIRICHLET && d->bc[1] == LBM_BC_DIRICHLET;
            const bool yp = d->bc[2] == LBM_BC_PERIODIC && d->bc[3] == LBM_BC_PERIODIC;
            const bool yw = d->bc[2] == LBM_BC_WALL && d->bc[3] == LBM_BC_WALL;
            const bool ys = d->bc[2] == LBM_BC_WALL && d->bc[3] == LBM_BC_SYMMETRY;
            if (!(xp || xio || xd) || !(yp || yw || ys))
                return fail(LBM_E_UNSUPPORTED,
                            "D2Q9_D2Q5: x periodic, inlet/outlet or fixed-T walls; y periodic, walls, "
                            "or wall + symmetry plane");
            if (xio && d->nx < 2) return fail(LBM_E_ARG, "inlet/outlet needs nx >= 2");
            if (xd && !(d->flags & LBM_FLAG_THERMAL))
                return fail(LBM_E_ARG, "fixed-temperature walls need the thermal field");
            if ((d->flags & ~(LBM_FLAG_FLOW | LBM_FLAG_THERMAL | LBM_FLAG_THERMAL_D2Q9)) != 0 ||
                (d->flags & (LBM_FLAG_FLOW | LBM_FLAG_THERMAL)) == 0)
                return fail(LBM_E_ARG, "flags must be a non-empty subset of FLOW | THERMAL (| THERMAL_D2Q9)");
            if ((d->flags & LBM_FLAG_THERMAL_D2Q9) && !(d->flags & LBM_FLAG_THERMAL))
                return fail(LBM_E_ARG, "THERMAL_D2Q9 needs THERMAL");
            l.npop = 9 + ((d->flags & LBM_FLAG_THERMAL) ? ((d->flags & LBM_FLAG_THERMAL_D2Q9) ? 9 : 5) : 0);
            break;
        }
        case LBM_D2Q9_PHASE: {
            const bool xp = d->bc[0] == LBM_BC_PERIODIC && d->bc[1] == LBM_BC_PERIODIC;
            const bool yp = d->bc[2] == LBM_BC_PERIODIC && d->bc[3] == LBM_BC_PERIODIC;
            const bool yw = d->bc[2] == LBM_BC_WALL && d->bc[3] == LBM_BC_WALL;
            if (!xp || !(yp || yw)) return fail(LBM_E_UNSUPPORTED, "PHASE: x periodic, y periodic or walls");
            l.npop = 18 + (d->prec != LBM_FP64 ? 1 : 0);
            break;
        }
        case LBM_D3Q19: {
            auto pair_ok = [](int a, int b) {
                return a == b && (a == LBM_BC_PERIODIC || a == LBM_BC_WALL);
            };
            if (!pair_ok(d->bc[0], d->bc[1]) || !pair_ok(d->bc[2], d->bc[3]) ||
                !pair_ok(d->bc_z[0], d->bc_z[1]))
                return fail(LBM_E_UNSUPPORTED, "D3Q19: each axis periodic or walls on both sides");
            if ((d->flags & ~LBM_FLAG_FLOW) != 0) return fail(LBM_E_ARG, "D3Q19 takes no flags but FLOW");
            l.npop = 19;
            break;
        }
        case LBM_D3Q19_PHASE: {
            auto pair_ok = [](int a, int b) {
                return a == b && (a == LBM_BC_PERIODIC || a == LBM_BC_WALL);
            };
            if (!pair_ok(d->bc[0], d->bc[1]) || !pair_ok(d->bc[2], d->bc[3]) ||
                !pair_ok(d->bc_z[0], d->bc_z[1]))
                return fail(LBM_E_UNSUPPORTED, "D3Q19_PHASE: each axis periodic or walls on both sides");
            if (d->flags != 0) return fail(LBM_E_ARG, "D3Q19_PHASE takes no flags");
            l.npop = 38 + (d->prec == LBM_FP32_DEV ? 1 : 0);
            break;
        }
        default:
            return fail(LBM_E_ARG, "unknown lattice");
    }
    {
        // one 256-thread workgroup per 64 x 4 tile (x 4 z planes for D3Q19):
        // the total thread count must fit the 32-bit launch grid
        const long long tiles = (long long)((d->nx + 63) / 64) * ((d->ny + 3) / 4) * nz * d->batch;
        if (tiles >= (1LL << 24)) return fail(LBM_E_ARG, "grid too large for the launch geometry");
    }
    // the PHASE states also carry (phi u) of the previous step: 2 or 3 planes
    l.nplanes = l.npop + (d->lattice == LBM_D2Q9_PHASE ? 2 : (d->lattice == LBM_D3Q19_PHASE ? 3 : 0));
    size_t off = 0;
    const size_t popbytes = align256((size_t)l.nplanes * l.P * l.es);
    l.offA = off; off += popbytes;
    l.offB = off; off += popbytes;
    l.offAux = off; off += align256((size_t)(d->nx + 2 * d->ny) * l.es);
    l.offStage = off; off += align256(8 * (size_t)l.P * sizeof(double));
    l.offPartial = off; off += align256((size_t)d->batch * 4 * kRedBlocks * sizeof(double));
    l.offSmall = off; off += align256((size_t)(3 * d->nx + 64 + 4 * d->batch) * sizeof(double));
    // D3Q19_PHASE: phi of the current state, recomputed before every step
    l.offPhi = off; off += d->lattice == LBM_D3Q19_PHASE ? align256((size_t)l.P * l.es) : 0;
    // the non-finite watch word (first step at which a check saw one)
    l.offWatch = off; off += 256;
    // D2Q9_PHASE: per-tile step counters and the error word of the
    // many-steps-per-launch kernel, in the buffer's last 256 bytes
    l.offFlags = off; off += d->lattice == LBM_D2Q9_PHASE ? kPersistFlagBytes : 0;
    l.total = off;
    *L = l;
    return LBM_OK;
}

lbm_status set_err(lbm_ctx* c, lbm_status st, const std::string& m) {
    c->err = m;
    return st;
}

lbm_status hip_fail(lbm_ctx* c, hipError_t e, const char* where) {
    return set_err(c, LBM_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

// Largest speed in a velocity component, in units of the lattice speed c = dx/dt;
// a NaN counts as above every limit.
double speed_over_c(const double* u, long long n, double dt_over_dx) {
    double m = 0.0;
    if (!u) return m;
    for (long long i = 0; i < n; ++i) {
        const double a = std::fabs(u[i]) * dt_over_dx;
        if (!(a <= m)) m = a;
    }
    return m;
}

// Speed limit of the warning, in units of c = dx/dt.  The equilibria are expanded
// to second order in u / c_s and their error grows as (u / c_s)^2; beyond 0.3 c
// (Ma = u / c_s = 0.52) a step is neither accurate nor reliably stable.
constexpr double kMachLimit = 0.3;

// Informational LBM_W_MACH when a given speed reaches kMachLimit of c.
lbm_status mach_status(lbm_ctx* c, double u_over_c, const char* what) {
    if (u_over_c <= kMachLimit) return LBM_OK;
    char m[200];
    std::snprintf(m, sizeof m, "%s: max |u| dt / dx = %.3g above %.2g (Ma = |u| / c_s = %.3g); "
                  "the second-order equilibria lose accuracy and stability", what, u_over_c,
                  kMachLimit, u_over_c * std::sqrt(3.0));
    return set_err(c, LBM_W_MACH, m);
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

uint64_t fnv(uint64_t h, const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

char* bufA(lbm_ctx* c) { return c->cur == 0 ? c->popA : c->popB; }
char* bufB(lbm_ctx* c) { return c->cur == 0 ? c->popB : c->popA; }

template <typename S>
S* aux_qw(lbm_ctx* c) { return (S*)c->aux; }
template <typename S>
S* aux_uin(lbm_ctx* c) { return (S*)c->aux + c->desc.nx; }
template <typename S>
S* aux_tin(lbm_ctx* c) { return (S*)c->aux + c->desc.nx + c->desc.ny; }

// wall-flux modulation of the step from time t dt
double flux_mod_at(const lbm_ctx* c, long long t) {
    return 1.0 + c->flux_amp * std::sin(c->flux_omega * (double)t * c->dt);
}
double flux_mod(const lbm_ctx* c) { return flux_mod_at(c, c->t); }

template <typename S>
hipError_t step_once(lbm_ctx* c) {
    const int lat = c->desc.lattice;
    S* a = (S*)bufA(c);
    S* b = (S*)bufB(c);
    if (lat == LBM_D3Q19) return launch_d3_step<S>(c->d3k, a, b, c->stream);
    if (lat == LBM_D3Q19_PHASE) return launch_p3_step<S>(c->p3k, a, b, (S*)c->phi3, c->stream);
    if (lat == LBM_D2Q9_D2Q5) {
        return launch_chan_step<S>(c->ck, a, b, aux_qw<S>(c), aux_uin<S>(c), aux_tin<S>(c),
                                   flux_mod(c), c->stream);
    }
    return launch_phase_step<S>(c->pk, a, b, c->desc.prec == LBM_FP32_DEV_ARITH64, c->stream);
}

// Whether the next two steps go through a two-step kernel (mode 2 takes it
// where the kernel covers the configuration).  Automatic mode takes it when
// its workgroups (one per row segment, x-tile and replica; two or three are
// resident per CU) fill the 256 CUs and, for rows in x-tiles, at least 90 %
// of the launched lanes hold stored columns; smaller or narrow grids keep
// the single-step kernel, whose tiles spread over more CUs.
bool use_tb2(const lbm_ctx* c) {
    if (c->fusion == 1 || c->tb2_seg < 1) return false;
    if (c->desc.lattice == LBM_D2Q9_D2Q5)
        return c->fusion == 2 || (c->fusion == 0 && chan_tb2_workgroups(c->ck, c->tb2_seg) >= 512 &&
                                  chan_tb2_lane_use(c->ck) >= 0.9);
    if (c->desc.lattice != LBM_D2Q9_PHASE) return false;
    if (c->fusion == 2) return true;
    return phase_tb2_workgroups(c->pk, c->tb2_seg) >= 512 && phase_tb2_lane_use(c->pk) >= 0.9;
}

// The many-steps kernel needs the grid split into at most kPersistMaxTiles
// tiles (of 512, 256 or 128 nodes) over all replicas, all resident at once.
bool phase_persist_fits_desc(const lbm_desc& d) {
    PhaseK k{};
    k.nx = d.nx;
    k.ny = d.ny;
    k.batch = d.batch;
    return phase_persist_fits(k);
}

// Under the caller's stream capture the steps take the single-step kernel
// (same states): the many-steps path ends with a synchronisation.
bool use_persist(const lbm_ctx* c) {
    if (c->desc.lattice != LBM_D2Q9_PHASE || c->fusion != 3 || !phase_persist_fits(c->pk))
        return false;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    return hipStreamIsCapturing(c->stream, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone;
}

// Clear the non-finite watch word (all ones: nothing seen) with a new state.
hipError_t reset_watch(lbm_ctx* c) {
    return hipMemsetAsync(c->watch, 0xff, sizeof(unsigned long long), c->stream);
}

// Zero the step counters and the error word: with the state (re)set no
// launch of the many-steps kernel is pending.
hipError_t reset_persist(lbm_ctx* c) {
    c->persist_epoch = 0;
    if (!c->persist_flags) return hipSuccess;
    return hipMemsetAsync(c->persist_flags, 0, kPersistFlagBytes, c->stream);
}

// n steps in launches of the many-steps kernel (at most kPersistChunk steps
// each), then one synchronisation to read the error word.
constexpr int kPersistChunk = 1 << 14;
template <typename S>
lbm_status step_persist(lbm_ctx* c, int n) {
    unsigned* err = c->persist_flags + kPersistMaxTiles;
    for (int s = 0; s < n;) {
        const int m = std::min(kPersistChunk, n - s);
        hipError_t e = launch_phase_persist<S>(c->pk, (S*)bufA(c), (S*)bufB(c), m, c->persist_epoch,
                                               c->persist_flags, err,
                                               c->desc.prec == LBM_FP32_DEV_ARITH64, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "many-steps kernel");
        c->persist_epoch += unsigned(m);
        c->cur ^= (m & 1);
        c->t += m;
        s += m;
    }
    unsigned herr = 0;
    hipError_t e = hipMemcpyAsync(&herr, err, sizeof(herr), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "many-steps kernel");
    if (herr) {
        c->has_state = false;
        return set_err(c, LBM_E_DEVICE, "many-steps kernel: a tile's wait for its neighbours timed "
                                        "out; the state is lost (reinitialise it)");
    }
    return LBM_OK;
}

// Enqueue m (1 or 2) steps, advancing the buffer parity and the step count;
// *swaps receives the number of buffer swaps made.
template <typename S>
hipError_t advance(lbm_ctx* c, int m, int* swaps) {
    *swaps = 0;
    if (m == 2 && use_tb2(c)) {
        hipError_t e =
            c->desc.lattice == LBM_D2Q9_D2Q5
                ? launch_chan_tb2<S>(c->ck, (const S*)bufA(c), (S*)bufB(c), aux_qw<S>(c),
                                     aux_uin<S>(c), aux_tin<S>(c), flux_mod_at(c, c->t),
                                     flux_mod_at(c, c->t + 1), c->tb2_seg, c->stream)
                : launch_phase_tb2<S>(c->pk, (const S*)bufA(c), (S*)bufB(c), c->tb2_seg,
                                      c->stream);
        if (e != hipSuccess) return e;
        c->cur ^= 1;
        c->t += 2;
        *swaps = 1;
        return hipSuccess;
    }
    for (int k = 0; k < m; ++k) {
        hipError_t e = step_once<S>(c);
        if (e != hipSuccess) return e;
        c->cur ^= 1;
        c->t += 1;
        ++*swaps;
    }
    return hipSuccess;
}

void drop_graphs(lbm_ctx* c) {
    for (hipGraphExec_t& g : c->step_graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

// A captured run of steps replays its kernel arguments unchanged, so it is
// only valid while no argument depends on the step count (the oscillating
// wall flux does) and while the caller's stream is not itself capturing.
bool graph_usable(lbm_ctx* c) {
    if (c->graph_steps <= 0) return false;
    if (c->desc.lattice == LBM_D2Q9_D2Q5 && c->ck.thermal && c->flux_amp != 0.0) return false;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(c->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
        return false;
    return true;
}

// Enqueue graph_steps steps as one graph launch.  The graph for the current
// buffer parity is captured on first use, with the buffer swaps it makes.
template <typename S>
hipError_t step_replay(lbm_ctx* c) {
    const int p0 = c->cur;
    hipGraphExec_t& ex = c->step_graph[p0];
    if (!ex) {
        hipError_t e = hipSuccess;
        if (!c->cap_stream) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return e;
        e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        const hipStream_t user = c->stream;
        const int cur0 = c->cur;
        c->stream = c->cap_stream;
        const long long t0 = c->t;
        hipError_t el = hipSuccess;
        int swaps = 0;
        for (int k = 0; k < c->graph_steps && el == hipSuccess; k += 2) {
            int sw = 0;
            el = advance<S>(c, 2, &sw);
            swaps += sw;
        }
        c->stream = user;
        c->cur = cur0;
        c->t = t0;
        c->graph_swaps[p0] = swaps;
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(c->cap_stream, &g);
        if (el != hipSuccess || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return el != hipSuccess ? el : e;
        }
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            ex = nullptr;
            return e;
        }
    }
    hipError_t e = hipGraphLaunch(ex, c->stream);
    if (e == hipSuccess) c->cur ^= (c->graph_swaps[p0] & 1);
    return e;
}

// Relaxation time from a diffusivity, tau = D / c_s^2 + dt/2 (Eq.
// eq_kinematic_viscosity and its thermal analogue), unless the caller gave
// tau itself (tau_given > 0).
double tau_or_nu(double tau_given, double D, double cs2, double dt) {
    return tau_given > 0 ? tau_given : D / cs2 + 0.5 * dt;
}

template <typename S>
hipError_t upload_aux(lbm_ctx* c, const lbm_params_si* p) {
    const int nx = c->desc.nx, ny = c->desc.ny;
    std::vector<S> h(nx + 2 * ny);
    const double cc = p->dx / p->dt;
    for (int x = 0; x < nx; ++x)
        h[x] = S(p->flux ? p->flux[x] * p->dt / (p->dx * p->rho_cp) : 0.0);
    for (int y = 0; y < ny; ++y) {
        h[nx + y] = S(p->inlet_u ? p->inlet_u[y] / cc : 0.0);
        h[nx + ny + y] = S(p->inlet_T ? p->inlet_T[y] - p->T_ref : 0.0);
    }
    hipError_t e = hipMemcpyAsync(c->aux, h.data(), h.size() * sizeof(S), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(c->stream);
}

}  // namespace

extern "C" {

lbm_status lbm_query_bytes(const lbm_desc* desc, size_t* bytes) {
    if (!bytes) return LBM_E_ARG;
    Layout L;
    lbm_status st = check_desc(desc, &L, nullptr);
    if (st != LBM_OK) return st;
    *bytes = L.total;
    return LBM_OK;
}

lbm_status lbm_create(const lbm_desc* desc, lbm_ctx** out) {
    if (!out) return LBM_E_ARG;
    Layout L;
    lbm_status st = check_desc(desc, &L, nullptr);
    if (st != LBM_OK) return st;
    if (!desc->dev_buf || desc->dev_buf_bytes < L.total) return LBM_E_ARG;
    if (((uintptr_t)desc->dev_buf & 255) != 0) return LBM_E_ARG;  // 256-byte aligned planes
    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return LBM_E_ARG;
    c->desc = *desc;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return LBM_E_DEVICE;
    }
    c->stream = (hipStream_t)desc->hip_stream;
    c->N = L.N;
    c->P = L.P;
    c->npop = L.npop;
    c->nplanes = L.nplanes;
    c->esize = L.es;
    char* base = (char*)desc->dev_buf;
    c->popA = base + L.offA;
    c->popB = base + L.offB;
    c->aux = base + L.offAux;
    c->staging = (double*)(base + L.offStage);
    c->partial = (double*)(base + L.offPartial);
    c->small = (double*)(base + L.offSmall);
    c->phi3 = base + L.offPhi;
    c->persist_flags = desc->lattice == LBM_D2Q9_PHASE ? (unsigned*)(base + L.offFlags) : nullptr;
    c->scratch = scratch_address(c->device);  // nullptr: lbm_reduce_noalloc reports it
    c->watch = (unsigned long long*)(base + L.offWatch);
    c->cur = 0;
    c->t = 0;
    c->has_params = c->has_state = false;
    c->has_record = false;
    *out = c;
    return LBM_OK;
}

void lbm_destroy(lbm_ctx* ctx) {
    if (!ctx) return;
    {
        DeviceGuard g(ctx->device);
        drop_graphs(ctx);
        if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    }
    delete ctx;
}

lbm_status lbm_set_graph_steps(lbm_ctx* c, int steps) {
    if (!c) return LBM_E_ARG;
    if (steps < 0 || steps > 4096 || (steps & 1))
        return set_err(c, LBM_E_ARG, "graph steps must be 0 or an even number up to 4096");
    if (steps != c->graph_steps) {
        DeviceGuard g(c->device);
        drop_graphs(c);
        c->graph_steps = steps;
    }
    return LBM_OK;
}

lbm_status lbm_set_step_fusion(lbm_ctx* c, int mode) {
    if (!c) return LBM_E_ARG;
    if (mode < 0 || mode > 3) return set_err(c, LBM_E_ARG, "fusion mode must be 0, 1, 2 or 3");
    if (mode == 3 && c->desc.lattice == LBM_D2Q9_PHASE && !phase_persist_fits_desc(c->desc))
        return set_err(c, LBM_E_UNSUPPORTED,
                       "many-steps kernel needs at most 16 tiles of 512 nodes over all replicas");
    if (mode == 2 && c->desc.lattice == LBM_D2Q9_PHASE && c->desc.prec == LBM_FP32_DEV_ARITH64)
        return set_err(c, LBM_E_UNSUPPORTED, "two-step kernel: not with FP64 arithmetic on FP32 storage");
    if (mode == 2 && c->desc.lattice == LBM_D2Q9_D2Q5 && c->has_params && !chan_tb2_fits(c->ck))
        return set_err(c, LBM_E_UNSUPPORTED,
                       "two-step channel kernel: needs both flow and temperature");
    if (mode != c->fusion) {
        DeviceGuard g(c->device);
        drop_graphs(c);
        c->fusion = mode;
    }
    return LBM_OK;
}

const char* lbm_last_error(const lbm_ctx* ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

long long lbm_time(const lbm_ctx* ctx) { return ctx ? ctx->t : -1; }

lbm_status lbm_set_params_SI(lbm_ctx* c, const lbm_params_si* p) {
    if (!c) return LBM_E_ARG;
    if (!p) return set_err(c, LBM_E_ARG, "params is NULL");
    if (!(p->dx > 0) || !(p->dt > 0)) return set_err(c, LBM_E_ARG, "dx and dt must be positive");
    const lbm_desc& d = c->desc;
    const double dx = p->dx, dt = p->dt, cc = dx / dt;
    ChanK ck{};
    PhaseK pk{};
    D1K dk{};
    D3K d3k{};
    P3K p3k{};
    AdjK ak{};
    c->fp32_forcing_share = 0.0;
    double alpha_eff = p->alpha;  // thermal diffusivity implied by tau_T, m^2/s
    if (d.lattice == LBM_D3Q19_PHASE) {
        const double cs2 = cc * cc / 3.0;
        p3k.nx = d.nx; p3k.ny = d.ny; p3k.nz = d.nz; p3k.batch = d.batch; p3k.P = c->P;
        p3k.bcx = d.bc[0] == LBM_BC_WALL;
        p3k.bcy = d.bc[2] == LBM_BC_WALL;
        p3k.bcz = d.bc_z[0] == LBM_BC_WALL;
        p3k.z_mrt = p->z_collision == LBM_MRT;
        p3k.visc_mode = p->visc_mode ? 1 : 0;
        if (!(p->rho_l > 0) || !(p->rho_g > 0)) return set_err(c, LBM_E_ARG, "densities must be positive");
        p3k.rho_l = p->rho_l;
        p3k.rho_g = p->rho_g;
        const double sc = dt / (dx * dx);
        if (p3k.visc_mode == 0) {
            if (!(p->nu_l > 0) || !(p->nu_g > 0)) return set_err(c, LBM_E_TAU, "tau not above dt/2 (nu <= 0)");
        } else {
            if (!(p->zeta_l > 0) || !(p->zeta_g > 0)) return set_err(c, LBM_E_TAU, "tau not above dt/2 (zeta <= 0)");
        }
        p3k.nuh_l = p->nu_l * sc; p3k.nuh_g = p->nu_g * sc;
        p3k.zh_l = p->zeta_l * sc; p3k.zh_g = p->zeta_g * sc;
        if (!(p->mobility > 0)) return set_err(c, LBM_E_TAU, "tau_phi not above dt/2 (mobility <= 0)");
        if (!(p->W > 0)) return set_err(c, LBM_E_ARG, "interface width must be positive");
        p3k.w_phi = dt / (p->mobility / cs2 + 0.5 * dt);  // M = (tau_phi - dt/2) c_s^2
        p3k.beta = 12.0 * p->sigma / p->W;
        p3k.kap6 = 6.0 * 1.5 * p->sigma * p->W / (dx * dx);  // 6 kappa / dx^2, kappa = 3 sigma W / 2
        p3k.fs_scale = 3.0 * dt * dt / (dx * dx);
        p3k.Fbt[0] = p->Fb[0] * dt * dt / dx;
        p3k.Fbt[1] = p->Fb[1] * dt * dt / dx;
        p3k.Fbt[2] = p->Fb_z * dt * dt / dx;
        p3k.dxW = dx / p->W;
        const double eps = p->normal_eps > 0 ? p->normal_eps
                                             : (d.prec == LBM_FP64 ? 1e-12 : 1e-6) / dx;
        p3k.Geps = eps * dx / 3.0;
        p3k.c = cc;
        p3k.cs2 = cs2;
    } else if (d.lattice == LBM_D3Q19) {
        const double cs2 = cc * cc / 3.0;
        d3k.nx = d.nx; d3k.ny = d.ny; d3k.nz = d.nz; d3k.batch = d.batch; d3k.P = c->P;
        d3k.bcx = d.bc[0] == LBM_BC_WALL;
        d3k.bcy = d.bc[2] == LBM_BC_WALL;
        d3k.bcz = d.bc_z[0] == LBM_BC_WALL;
        if (!(p->rho_ref > 0)) return set_err(c, LBM_E_ARG, "rho_ref must be positive");
        const double tau = tau_or_nu(p->tau, p->nu, cs2, dt);  // Eq. eq_kinematic_viscosity
        if (!(tau > 0.5 * dt)) return set_err(c, LBM_E_TAU, "tau not above dt/2");
        d3k.rho_ref = p->rho_ref;
        const double wn = dt / tau;
        if (p->flow_collision == LBM_MRT) {
            // Sec. 3 in the 3D basis: e, eps free; stresses at 1/tau; q (and the
            // third-order m) at (3/dt)(2/dt - w)/(3/dt - w); pi at 1/dt -- all times dt
            const double wq = 3.0 * (2.0 - wn) / (3.0 - wn);
            const double we = p->omega_e > 0 ? p->omega_e * dt : 1.0;
            const double wpe = p->omega_eps > 0 ? p->omega_eps * dt : 1.0;
            const double L[19] = {0, we, wpe, 0, wq, 0, wq, 0, wq, wn, 1.0, wn, 1.0,
                                  wn, wn, wn, wq, wq, wq};
            for (int q = 0; q < 19; ++q) d3k.L[q] = L[q];
        } else {
            // BGK: every non-conserved moment at dt/tau
            for (int q = 0; q < 19; ++q) d3k.L[q] = (q == 0 || q == 3 || q == 5 || q == 7) ? 0.0 : wn;
        }
        d3k.Ft[0] = p->Fb[0] * dt * dt / dx;
        d3k.Ft[1] = p->Fb[1] * dt * dt / dx;
        d3k.Ft[2] = p->Fb_z * dt * dt / dx;
        d3k.c = cc;
    } else if (d.lattice == LBM_D1Q2 || d.lattice == LBM_D1Q3) {
        const double cs2 = d.lattice == LBM_D1Q2 ? cc * cc : cc * cc / 3.0;
        if (!(p->rho_cp > 0)) return set_err(c, LBM_E_ARG, "rho_cp must be positive");
        const double tau = tau_or_nu(p->tau_T, p->alpha, cs2, dt);
        if (!(tau > 0.5 * dt)) return set_err(c, LBM_E_TAU, "tau_T not above dt/2");
        alpha_eff = (tau - 0.5 * dt) * cs2;
        dk.n = d.nx;
        dk.q = d.lattice == LBM_D1Q2 ? 2 : 3;
        dk.w_tau = dt / tau;
        dk.qdt = p->qvol / p->rho_cp * dt;
        dk.ufac = 0.0;
        dk.T0 = p->T_wall[0];
        dk.TL = p->T_wall[1];
    } else if (d.lattice == LBM_D2Q9_D2Q5) {
        const double cs2 = cc * cc / 3.0;
        ck.nx = d.nx; ck.ny = d.ny; ck.batch = d.batch; ck.P = c->P; ck.npl = c->nplanes;
        ck.bcx = d.bc[0] == LBM_BC_VEL_INLET ? 1 : (d.bc[0] == LBM_BC_DIRICHLET ? 2 : 0);
        ck.bcy = d.bc[2] == LBM_BC_WALL ? (d.bc[3] == LBM_BC_SYMMETRY ? 2 : 1) : 0;
        ck.flow = (d.flags & LBM_FLAG_FLOW) ? 1 : 0;
        ck.thermal = (d.flags & LBM_FLAG_THERMAL) ? 1 : 0;
        ck.tq = (d.flags & LBM_FLAG_THERMAL_D2Q9) ? 9 : 5;
        ck.flow_mrt = p->flow_collision == LBM_MRT;
        ck.thermal_mrt = p->thermal_collision == LBM_MRT;
        if (!(p->rho_ref > 0)) return set_err(c, LBM_E_ARG, "rho_ref must be positive");
        ck.rho_ref = p->rho_ref;
        if (ck.flow) {
            const double tau = tau_or_nu(p->tau, p->nu, cs2, dt);  // Eq. eq_kinematic_viscosity
            if (!(tau > 0.5 * dt)) return set_err(c, LBM_E_TAU, "tau not above dt/2");
            const double wn = dt / tau;
            // dimensional w_q = (3/dt)(2/dt - w_nu)/(3/dt - w_nu) (Sec. 3), times dt
            const double wq = 3.0 * (2.0 - wn) / (3.0 - wn);
            const double we = p->omega_e > 0 ? p->omega_e * dt : 1.0;
            const double wpe = p->omega_eps > 0 ? p->omega_eps * dt : 1.0;
            const double Lf[9] = {0, we, wpe, 0, wq, 0, wq, wn, wn};
            for (int q = 0; q < 9; ++q) ck.Lf[q] = Lf[q];
            // derivatives with respect to tau of w_nu dt = dt/tau and w_q dt
            const double dwn = -dt / (tau * tau);
            const double dwq = 3.0 * dt / (tau * tau * (3.0 - wn) * (3.0 - wn));
            const double dL[9] = {0, 0, 0, 0, dwq, 0, dwq, dwn, dwn};
            for (int q = 0; q < 9; ++q) ak.dLf[q] = ck.flow_mrt ? dL[q] : (q == 7 ? dwn : 0.0);
        }
        ck.Ft[0] = p->Fb[0] * dt * dt / dx;
        ck.Ft[1] = p->Fb[1] * dt * dt / dx;
        if (ck.thermal) {
            const double tauT = tau_or_nu(p->tau_T, p->alpha, cs2, dt);
            if (!(tauT > 0.5 * dt)) return set_err(c, LBM_E_TAU, "tau_T not above dt/2");
            if (!(p->rho_cp > 0)) return set_err(c, LBM_E_ARG, "rho_cp must be positive");
            alpha_eff = (tauT - 0.5 * dt) * cs2;
            const double wT = dt / tauT, dwT = -dt / (tauT * tauT);
            // MRT: the fluxes j relax at dt/tau_T, the conserved T not at all, the
            // rest at 1 (Lambda_T,dim of Sec. 3 on D2Q9; its two-rate analogue on D2Q5)
            for (int q = 0; q < ck.tq; ++q) {
                const bool j = ck.tq == 9 ? (q == 3 || q == 5) : (q == 1 || q == 2);
                ck.Lt[q] = ck.thermal_mrt ? (j ? wT : (q == 0 ? 0.0 : 1.0)) : wT;
                if (q < 5) ak.dLt[q] = (ck.thermal_mrt && !j) ? 0.0 : dwT;
            }
            ak.qgrad = dt / (dx * p->rho_cp);
            ck.qdt = p->qvol / p->rho_cp * dt;
        }
        ck.c = cc;
        ck.T_ref = p->T_ref;
        ck.Tw[0] = p->T_wall[0] - p->T_ref;
        ck.Tw[1] = p->T_wall[1] - p->T_ref;
        // Boussinesq force -rho_ref beta (T - T_ref) g (Eq. buoyancy_force), per kelvin
        ck.buoy = p->beta_T != 0.0 && (p->gravity[0] != 0.0 || p->gravity[1] != 0.0);
        if (ck.buoy && !ck.thermal)
            return set_err(c, LBM_E_ARG, "the Boussinesq force needs the thermal field");
        ck.Bt[0] = -p->rho_ref * p->beta_T * p->gravity[0] * dt * dt / dx;
        ck.Bt[1] = -p->rho_ref * p->beta_T * p->gravity[1] * dt * dt / dx;
    } else {
        const double cs2 = cc * cc / 3.0;
        pk.nx = d.nx; pk.ny = d.ny; pk.batch = d.batch; pk.P = c->P;
        pk.bcy = d.bc[2] == LBM_BC_WALL ? 1 : 0;
        pk.z_mrt = p->z_collision == LBM_MRT;
        pk.qy_printed = p->qy_printed ? 1 : 0;
        pk.visc_mode = p->visc_mode ? 1 : 0;
        if (!(p->rho_l > 0) || !(p->rho_g > 0)) return set_err(c, LBM_E_ARG, "densities must be positive");
        pk.rho_l = p->rho_l;
        pk.rho_g = p->rho_g;
        const double s = dt / (dx * dx);
        if (pk.visc_mode == 0) {
            if (!(p->nu_l > 0) || !(p->nu_g > 0)) return set_err(c, LBM_E_TAU, "tau not above dt/2 (nu <= 0)");
        } else {
            if (!(p->zeta_l > 0) || !(p->zeta_g > 0)) return set_err(c, LBM_E_TAU, "tau not above dt/2 (zeta <= 0)");
        }
        pk.nuh_l = p->nu_l * s; pk.nuh_g = p->nu_g * s;
        pk.zh_l = p->zeta_l * s; pk.zh_g = p->zeta_g * s;
        if (!(p->mobility > 0)) return set_err(c, LBM_E_TAU, "tau_phi not above dt/2 (mobility <= 0)");
        if (!(p->W > 0)) return set_err(c, LBM_E_ARG, "interface width must be positive");
        pk.w_phi = dt / (p->mobility / cs2 + 0.5 * dt);  // M = (tau_phi - dt/2) c_s^2
        pk.beta = 12.0 * p->sigma / p->W;                 // beta = 12 sigma / W
        const double kappa = 1.5 * p->sigma * p->W;       // kappa = 3 sigma W / 2
        pk.kap6 = 6.0 * kappa / (dx * dx);
        pk.fs_scale = 3.0 * dt * dt / (dx * dx);
        pk.Fbt[0] = p->Fb[0] * dt * dt / dx;
        pk.Fbt[1] = p->Fb[1] * dt * dt / dx;
        pk.dxW = dx / p->W;
        const double eps = p->normal_eps > 0 ? p->normal_eps
                                             : (d.prec == LBM_FP64 ? 1e-12 : 1e-6) / dx;
        pk.Geps = eps * dx / 3.0;
        pk.c = cc;
        pk.cs2 = cs2;
        // FP32 forcing guard.  A body force builds the flow up over the
        // slowest viscous mode, whose share of the remaining change per step
        // is nu dt k^2 (k = pi / H between walls H apart, 2 pi / L for a period
        // L).  Once that share is below FP32's resolution, FP32 arithmetic
        // rounds part of every step's force increment away and long runs
        // drift (the layered channel at the paper's finest grid: 9-12 %).
        if (d.prec == LBM_FP32_DEV && (p->Fb[0] != 0.0 || p->Fb[1] != 0.0)) {
            const double nu_min = pk.visc_mode == 0
                                      ? std::min(p->nu_l, p->nu_g)
                                      : std::min(p->zeta_l / p->rho_l, p->zeta_g / p->rho_g);
            const double kw = pk.bcy ? M_PI / (d.ny * dx) : 2.0 * M_PI / (std::max(d.nx, d.ny) * dx);
            c->fp32_forcing_share = nu_min * dt * kw * kw;
        }
    }
    c->ck = ck;
    c->pk = pk;
    c->tb2_seg = 0;
    if (d.lattice == LBM_D2Q9_PHASE && phase_tb2_fits(pk)) {
        DeviceGuard g(c->device);
        c->tb2_seg = d.prec == LBM_FP64                ? phase_tb2_seg<double>(pk)
                     : d.prec == LBM_FP32_DEV_ARITH64 ? 0  // the two-step kernel computes in S
                                                       : phase_tb2_seg<float>(pk);
    }
    if (d.lattice == LBM_D2Q9_D2Q5 && chan_tb2_fits(ck)) {
        DeviceGuard g(c->device);
        c->tb2_seg = d.prec == LBM_FP64 ? chan_tb2_seg<double>(ck) : chan_tb2_seg<float>(ck);
    }
    c->dk = dk;
    c->d3k = d3k;
    c->p3k = p3k;
    c->ak = ak;
    c->cs2 = cc * cc / 3.0;
    c->has_record = false;
    c->sp = *p;
    c->sp.flux = c->sp.inlet_u = c->sp.inlet_T = nullptr;
    c->flux_amp = p->flux_amp;
    c->flux_omega = p->flux_omega;
    c->dt = dt;
    c->dx = dx;
    c->rho_cp = p->rho_cp;
    c->k_cond = p->rho_cp * alpha_eff;
    // hydraulic diameter 2H; with a symmetry plane the grid is half of H
    c->Dh = 2.0 * d.ny * dx * (d.lattice == LBM_D2Q9_D2Q5 && d.bc[3] == LBM_BC_SYMMETRY ? 2.0 : 1.0);
    uint64_t h = 1469598103934665603ull;
    h = fnv(h, &d.lattice, sizeof(int) * 5);
    h = fnv(h, d.bc, sizeof d.bc);
    h = fnv(h, &d.flags, sizeof(int));
    h = fnv(h, &ck, sizeof ck);
    h = fnv(h, &pk, sizeof pk);
    h = fnv(h, &dk, sizeof dk);
    h = fnv(h, &d.nz, sizeof d.nz);
    h = fnv(h, d.bc_z, sizeof d.bc_z);
    h = fnv(h, &d3k, sizeof d3k);
    h = fnv(h, &p3k, sizeof p3k);
    c->hash = h;
    DeviceGuard g(c->device);
    if (d.lattice == LBM_D2Q9_D2Q5) {
        hipError_t e = d.prec == LBM_FP64 ? upload_aux<double>(c, p) : upload_aux<float>(c, p);
        if (e != hipSuccess) return hip_fail(c, e, "upload of flux/inlet arrays");
    }
    {
        DeviceGuard g(c->device);
        drop_graphs(c);  // captured kernel arguments are stale now
    }
    c->has_params = true;
    int warn = 0;
    std::string msg;
    if (c->fp32_forcing_share > 0.0 && c->fp32_forcing_share < std::ldexp(1.0, -23)) {
        char m[256];
        std::snprintf(m, sizeof m,
                      "parameters set; the slowest viscous mode changes by %.2e of itself per step, "
                      "below FP32 resolution: FP32 arithmetic rounds the body-force increments of "
                      "long runs (LBM_FP32_DEV_ARITH64 keeps them)", c->fp32_forcing_share);
        warn |= LBM_W_FP32_FORCING;
        msg = m;
    }
    if (d.lattice == LBM_D2Q9_D2Q5 && (d.flags & LBM_FLAG_FLOW) && d.bc[0] == LBM_BC_VEL_INLET &&
        mach_status(c, speed_over_c(p->inlet_u, d.ny, dt / dx), "inlet profile") != LBM_OK) {
        warn |= LBM_W_MACH;
        msg = msg.empty() ? c->err : msg + "; " + c->err;
    }
    if (warn) set_err(c, (lbm_status)warn, msg);
    return (lbm_status)warn;
}

lbm_status lbm_init_fields(lbm_ctx* c, const double* rho_or_p, const double* ux, const double* uy,
                           const double* T, const double* phi) {
    if (!c) return LBM_E_ARG;
    if (!c->has_params) return set_err(c, LBM_E_STATE, "lbm_set_params_SI must come first");
    const lbm_desc& d = c->desc;
    const long long N = c->N, P = c->P;
    const bool d1 = d.lattice == LBM_D1Q2 || d.lattice == LBM_D1Q3;
    if (d1 && !T) return set_err(c, LBM_E_ARG, "1D lattices need T");
    if (d.lattice == LBM_D2Q9_D2Q5 && !rho_or_p) return set_err(c, LBM_E_ARG, "rho is required");
    if (d.lattice == LBM_D2Q9_PHASE && !phi) return set_err(c, LBM_E_ARG, "phi is required");
    if (d.lattice == LBM_D3Q19 || d.lattice == LBM_D3Q19_PHASE)
        return set_err(c, LBM_E_ARG, "3D lattices are initialised by lbm_init_fields3d");
    DeviceGuard g(c->device);
    std::vector<double> host(5 * (size_t)N, 0.0);
    auto put = [&](int slot, const double* src, double dflt) {
        for (long long n = 0; n < N; ++n) host[slot * (size_t)N + n] = src ? src[n] : dflt;
    };
    put(0, d.lattice == LBM_D2Q9_PHASE ? rho_or_p : (d1 ? T : rho_or_p), 0.0);
    put(1, ux, 0.0);
    put(2, uy, 0.0);
    put(3, T, c->sp.T_ref);
    put(4, phi, 0.0);
    for (int s = 0; s < 5; ++s) {
        hipError_t e = hipMemcpyAsync(c->staging + s * P, host.data() + s * (size_t)N,
                                      N * sizeof(double), hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "field upload");
    }
    c->cur = 0;
    hipError_t e = reset_persist(c);
    if (e == hipSuccess) e = reset_watch(c);
    if (e != hipSuccess) return hip_fail(c, e, "step counter reset");
    if (d1) {
        e = launch_d1_init(c->dk, c->staging, (double*)c->popA, c->stream);
    } else if (d.lattice == LBM_D2Q9_D2Q5) {
        if (d.prec == LBM_FP64)
            e = launch_chan_init<double>(c->ck, c->staging, (double*)c->popA, c->stream);
        else
            e = launch_chan_init<float>(c->ck, c->staging, (float*)c->popA, c->stream);
    } else {
        if (d.prec == LBM_FP64)
            e = launch_phase_init<double>(c->pk, c->staging, (double*)c->popA, c->stream);
        else
            e = launch_phase_init<float>(c->pk, c->staging, (float*)c->popA, c->stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "init kernel");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "init");
    c->t = 0;
    c->has_state = true;
    const double r = c->dt / c->dx;
    return mach_status(c, std::max(speed_over_c(ux, N, r), speed_over_c(uy, N, r)),
                       "initial velocity");
}

lbm_status lbm_init_fields3d(lbm_ctx* c, const double* rho_or_p, const double* ux,
                             const double* uy, const double* uz, const double* phi) {
    if (!c) return LBM_E_ARG;
    const int lat = c->desc.lattice;
    if (lat != LBM_D3Q19 && lat != LBM_D3Q19_PHASE)
        return set_err(c, LBM_E_ARG, "lbm_init_fields3d is for the 3D lattices");
    if (!c->has_params) return set_err(c, LBM_E_STATE, "lbm_set_params_SI must come first");
    if (lat == LBM_D3Q19 && !rho_or_p) return set_err(c, LBM_E_ARG, "rho is required");
    if (lat == LBM_D3Q19_PHASE && !phi) return set_err(c, LBM_E_ARG, "phi is required");
    const long long N = c->N, P = c->P;
    DeviceGuard g(c->device);
    std::vector<double> host((size_t)N);
    // staging slots: rho 0 or p 1, ux 2, uy 3, phi 5, uz 7
    const double* src[5] = {rho_or_p, ux, uy, uz, phi};
    const int slot[5] = {lat == LBM_D3Q19 ? 0 : 1, 2, 3, 7, 5};
    for (int k = 0; k < 5; ++k) {
        for (long long n = 0; n < N; ++n) host[n] = src[k] ? src[k][n] : 0.0;
        hipError_t e = hipMemcpyAsync(c->staging + slot[k] * P, host.data(), N * sizeof(double),
                                      hipMemcpyHostToDevice, c->stream);
        // the host vector is reused: wait for each copy
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "field upload");
    }
    c->cur = 0;
    const bool f64 = c->desc.prec == LBM_FP64;
    hipError_t e = reset_watch(c);
    if (e != hipSuccess) return hip_fail(c, e, "watch reset");
    if (lat == LBM_D3Q19)
        e = f64 ? launch_d3_init<double>(c->d3k, c->staging, (double*)c->popA, c->stream)
                : launch_d3_init<float>(c->d3k, c->staging, (float*)c->popA, c->stream);
    else
        e = f64 ? launch_p3_init<double>(c->p3k, c->staging, (double*)c->popA, c->stream)
                : launch_p3_init<float>(c->p3k, c->staging, (float*)c->popA, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "init kernel");
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "init");
    c->t = 0;
    c->has_state = true;
    const double r = c->dt / c->dx;
    return mach_status(c, std::max({speed_over_c(ux, N, r), speed_over_c(uy, N, r),
                                    speed_over_c(uz, N, r)}),
                       "initial velocity");
}

}  // extern "C"

namespace {

// n steps of the current kernel choice (the body of lbm_step).
lbm_status step_run(lbm_ctx* c, int n) {
    const int lat = c->desc.lattice;
    if (lat == LBM_D1Q2 || lat == LBM_D1Q3) {
        if (n == 0) return LBM_OK;
        hipError_t e = launch_d1(c->dk, (double*)c->popA, n, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "d1 kernel");
        c->t += n;
        return LBM_OK;
    }
    const bool f64 = c->desc.prec == LBM_FP64;
    if (n > 0 && use_persist(c)) return f64 ? step_persist<double>(c, n) : step_persist<float>(c, n);
    int s = 0;
    if (n >= 2 * c->graph_steps && graph_usable(c)) {
        for (; s + c->graph_steps <= n; s += c->graph_steps) {
            hipError_t e = f64 ? step_replay<double>(c) : step_replay<float>(c);
            if (e != hipSuccess) return hip_fail(c, e, "step graph");
            c->t += c->graph_steps;
        }
    }
    while (s < n) {
        const int m = n - s >= 2 ? 2 : 1;
        int sw = 0;
        hipError_t e = f64 ? advance<double>(c, m, &sw) : advance<float>(c, m, &sw);
        if (e != hipSuccess) return hip_fail(c, e, "step kernel");
        s += m;
    }
    return LBM_OK;
}

// The non-finite check of the current state (every node value of every
// state plane), recorded against the step count.
hipError_t watch_now(lbm_ctx* c) {
    const char* a = (c->desc.lattice == LBM_D1Q2 || c->desc.lattice == LBM_D1Q3) ? c->popA : bufA(c);
    const bool blocked = node_blocked(c->desc.lattice);
    if (c->desc.prec == LBM_FP64)
        return launch_nonfinite_watch<double>((const double*)a, c->P, c->N, c->nplanes, blocked,
                                              (unsigned long long)c->t, c->watch, c->stream);
    return launch_nonfinite_watch<float>((const float*)a, c->P, c->N, c->nplanes, blocked,
                                         (unsigned long long)c->t, c->watch, c->stream);
}

}  // namespace

extern "C" {

// n steps; every time the step count reaches a multiple of watch_every, the
// state is checked for non-finite values (not while the caller captures the
// stream: a captured check would replay a stale step count).
lbm_status lbm_step(lbm_ctx* c, int n) {
    if (!c) return LBM_E_ARG;
    if (n < 0) return set_err(c, LBM_E_ARG, "n must be >= 0");
    if (!c->has_state) return set_err(c, LBM_E_STATE, "no state: call lbm_init_fields or lbm_load_state");
    DeviceGuard g(c->device);
    const long long K = c->watch_every;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const bool capturing =
        hipStreamIsCapturing(c->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone;
    if (K <= 0 || capturing) return step_run(c, n);
    long long left = n;
    while (left > 0) {
        const long long to_mark = K - (c->t % K);  // steps to the next multiple of K
        const int m = (int)std::min(left, to_mark);
        lbm_status st = step_run(c, m);
        if (st != LBM_OK) return st;
        left -= m;
        if (c->t % K == 0) {
            hipError_t e = watch_now(c);
            if (e != hipSuccess) return hip_fail(c, e, "non-finite watch");
        }
    }
    return LBM_OK;
}

lbm_status lbm_set_nonfinite_check(lbm_ctx* c, int every) {
    if (!c) return LBM_E_ARG;
    if (every < 0) return set_err(c, LBM_E_ARG, "check interval must be >= 0");
    c->watch_every = every;
    return LBM_OK;
}

lbm_status lbm_first_nonfinite_step(lbm_ctx* c, long long* step) {
    if (!c) return LBM_E_ARG;
    if (!step) return set_err(c, LBM_E_ARG, "step is NULL");
    if (!c->has_state) return set_err(c, LBM_E_STATE, "no state");
    DeviceGuard g(c->device);
    unsigned long long w = ~0ull;
    hipError_t e = hipMemcpyAsync(&w, c->watch, sizeof w, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "non-finite watch");
    *step = w == ~0ull ? -1 : (long long)w;
    if (w == ~0ull) return LBM_OK;
    char m[160];
    std::snprintf(m, sizeof m, "non-finite state seen by the check at step %llu (checks every %d steps)",
                  w, c->watch_every);
    return set_err(c, LBM_E_NONFINITE, m);
}

lbm_status lbm_macros(lbm_ctx* c, unsigned mask, double* out, int out_on_device) {
    if (!c) return LBM_E_ARG;
    if (!out) return set_err(c, LBM_E_ARG, "out is NULL");
    if (!c->has_state) return set_err(c, LBM_E_STATE, "no state");
    const int lat = c->desc.lattice;
    unsigned avail;
    if (lat == LBM_D2Q9_D2Q5) avail = LBM_M_RHO | LBM_M_UX | LBM_M_UY | (c->ck.thermal ? LBM_M_T : 0u);
    else if (lat == LBM_D2Q9_PHASE) avail = LBM_M_RHO | LBM_M_P | LBM_M_UX | LBM_M_UY | LBM_M_PHI | LBM_M_MU;
    else if (lat == LBM_D3Q19) avail = LBM_M_RHO | LBM_M_UX | LBM_M_UY | LBM_M_UZ;
    else if (lat == LBM_D3Q19_PHASE)
        avail = LBM_M_RHO | LBM_M_P | LBM_M_UX | LBM_M_UY | LBM_M_UZ | LBM_M_PHI | LBM_M_MU;
    else avail = LBM_M_T;
    if (mask == 0 || (mask & ~avail)) return set_err(c, LBM_E_ARG, "field not available for this lattice");
    DeviceGuard g(c->device);
    const long long P = c->P, N = c->N;
    hipError_t e;
    const bool f64 = c->desc.prec == LBM_FP64;
    char* a = bufA(c);
    if (lat == LBM_D3Q19) {
        if (f64) e = launch_d3_macros<double>(c->d3k, (double*)a, c->staging, c->stream);
        else e = launch_d3_macros<float>(c->d3k, (float*)a, c->staging, c->stream);
    } else if (lat == LBM_D3Q19_PHASE) {
        if (f64) e = launch_p3_macros<double>(c->p3k, (double*)a, (double*)c->phi3, c->staging, c->stream);
        else e = launch_p3_macros<float>(c->p3k, (float*)a, (float*)c->phi3, c->staging, c->stream);
    } else if (lat == LBM_D2Q9_D2Q5) {
        if (f64) e = launch_chan_macros<double>(c->ck, (double*)a, c->staging, c->stream);
        else e = launch_chan_macros<float>(c->ck, (float*)a, c->staging, c->stream);
    } else if (lat == LBM_D2Q9_PHASE) {
        if (f64) e = launch_phase_macros<double>(c->pk, (double*)a, c->staging, c->stream);
        else e = launch_phase_macros<float>(c->pk, (float*)a, c->staging, c->stream);
    } else {
        e = launch_d1_macros(c->dk, (double*)c->popA, c->staging, P, c->stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "macros kernel");
    int k = 0;
    for (int bit = 0; bit < 8; ++bit) {
        if (!(mask & (1u << bit))) continue;
        e = hipMemcpyAsync(out + (size_t)k * N, c->staging + bit * P, N * sizeof(double),
                           out_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "macros copy");
        ++k;
    }
    if (!out_on_device) {
        e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "macros");
    }
    return LBM_OK;
}

lbm_status lbm_reduce(lbm_ctx* c, unsigned mask, double* out) {
    if (!c) return LBM_E_ARG;
    if (!out) return set_err(c, LBM_E_ARG, "out is NULL");
    if (!c->has_state) return set_err(c, LBM_E_STATE, "no state");
    if (mask == 0 || (mask & ~15u)) return set_err(c, LBM_E_ARG, "bad reduction mask");
    DeviceGuard g(c->device);
    const int lat = c->desc.lattice;
    const int batch = c->desc.batch;
    double* res = c->small + 3 * c->desc.nx + 64;
    hipError_t e;
    if (c->desc.prec == LBM_FP64)
        e = launch_reduce<double>(lat, c->ck, c->pk, c->dk, c->d3k, c->p3k, (const double*)bufA(c), c->npop,
                                  c->partial, res, c->stream);
    else
        e = launch_reduce<float>(lat, c->ck, c->pk, c->dk, c->d3k, c->p3k, (const float*)bufA(c), c->npop,
                                 c->partial, res, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "reduce kernel");
    std::vector<double> h(4 * (size_t)batch);
    e = hipMemcpyAsync(h.data(), res, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "reduce");
    int k = 0;
    bool nonfinite = false;
    for (int f = 0; f < 4; ++f) {
        for (int b = 0; b < batch; ++b) {
            if (h[b * 4 + 3] > 0) nonfinite = true;
            if (mask & (1u << f)) out[(size_t)k * batch + b] = h[b * 4 + f];
        }
        if (mask & (1u << f)) ++k;
    }
    if (nonfinite) {
        unsigned long long w = ~0ull;
        if (hipMemcpy(&w, c->watch, sizeof w, hipMemcpyDeviceToHost) == hipSuccess && w != ~0ull) {
            char m[160];
            std::snprintf(m, sizeof m, "non-finite populations in the state (first seen by the "
                                       "in-step check at step %llu)", w);
            return set_err(c, LBM_E_NONFINITE, m);
        }
        return set_err(c, LBM_E_NONFINITE, "non-finite populations in the state");
    }
    return LBM_OK;
}

lbm_status lbm_reduce_noalloc(lbm_ctx* c, unsigned mask, double* out) {
    if (!c) return LBM_E_ARG;
    if (!out) return set_err(c, LBM_E_ARG, "out is NULL");
    if (!c->has_state) return set_err(c, LBM_E_STATE, "no state");
    if (mask == 0 || (mask & ~15u)) return set_err(c, LBM_E_ARG, "bad reduction mask");
    const int batch = c->desc.batch;
    if (batch > kNoAllocMaxBatch)
        return set_err(c, LBM_E_ARG, "lbm_reduce_noalloc: at most 1024 replicas (static scratch)");
    if (!c->scratch)
        return set_err(c, LBM_E_DEVICE, "lbm_reduce_noalloc: no address for the static scratch");
    DeviceGuard g(c->device);
    const int lat = c->desc.lattice;
    double* partial = c->scratch;
    double* res = c->scratch + (size_t)batch * 4 * kRedBlocks;
    hipError_t e;
    if (c->desc.prec == LBM_FP64)
        e = launch_reduce<double>(lat, c->ck, c->pk, c->dk, c->d3k, c->p3k, (const double*)bufA(c),
                                  c->npop, partial, res, c->stream);
    else
        e = launch_reduce<float>(lat, c->ck, c->pk, c->dk, c->d3k, c->p3k, (const float*)bufA(c),
                                 c->npop, partial, res, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "reduce kernel");
    double h[4 * kNoAllocMaxBatch];  // host copy on the stack: no allocation anywhere
    e = hipMemcpyAsync(h, res, 4 * (size_t)batch * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "reduce");
    int k = 0;
    bool nonfinite = false;
    for (int f = 0; f < 4; ++f) {
        for (int b = 0; b < batch; ++b) {
            if (h[b * 4 + 3] > 0) nonfinite = true;
            if (mask & (1u << f)) out[(size_t)k * batch + b] = h[b * 4 + f];
        }
        if (mask & (1u << f)) ++k;
    }
    if (nonfinite) return set_err(c, LBM_E_NONFINITE, "non-finite populations in the state");
    return LBM_OK;
}

lbm_status lbm_nusselt(lbm_ctx* c, int x_dev, double* Tb, double* Tw, double* Nu, double* nu_mean,
                       double* T_out) {
    if (!c) return LBM_E_ARG;
    if (c->desc.lattice != LBM_D2Q9_D2Q5 || !c->ck.flow || !c->ck.thermal || !c->ck.bcy)
        return set_err(c, LBM_E_UNSUPPORTED, "Nusselt needs D2Q9_D2Q5 with flow, thermal and walls");
    if (!c->has_state) return set_err(c, LBM_E_STATE, "no state");
    const int nx = c->desc.nx;
    if (x_dev < 0 || x_dev >= nx) return set_err(c, LBM_E_ARG, "x_dev out of range");
    DeviceGuard g(c->device);
    double* dTb = c->small;
    double* dTw = c->small + nx;
    double* dNu = c->small + 2 * nx;
    double* dres = c->small + 3 * nx;
    const double qsi = c->dx * c->rho_cp / c->dt * flux_mod(c);
    hipError_t e;
    if (c->desc.prec == LBM_FP64) {
        const double* a = (const double*)bufA(c);
        e = launch_nusselt<double>(c->ck, a, aux_qw<double>(c), qsi, c->Dh, c->k_cond, c->dx, x_dev,
                                   dTb, dTw, dNu, dres, c->stream);
    } else {
        const float* a = (const float*)bufA(c);
        e = launch_nusselt<float>(c->ck, a, aux_qw<float>(c), qsi, c->Dh, c->k_cond, c->dx, x_dev,
                                  dTb, dTw, dNu, dres, c->stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "nusselt kernel");
    std::vector<double> h(3 * (size_t)nx + 2);
    e = hipMemcpyAsync(h.data(), c->small, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "nusselt");
    if (Tb) std::memcpy(Tb, h.data(), nx * sizeof(double));
    if (Tw) std::memcpy(Tw, h.data() + nx, nx * sizeof(double));
    if (Nu) std::memcpy(Nu, h.data() + 2 * nx, nx * sizeof(double));
    if (nu_mean) *nu_mean = h[3 * nx];
    if (T_out) *T_out = h[3 * nx + 1];
    return LBM_OK;
}

}  // extern "C"

// ---- discrete adjoint ------------------------------------------------------
namespace {

struct RecLayout {
    size_t state, offCk, offTape, offLam, offDq, offAcc, offGrad, total;
    int nseg, tiles;
};

lbm_status rec_layout(const lbm_ctx* c, int nsteps, int K, RecLayout* R, std::string* err) {
    const lbm_desc& d = c->desc;
    auto fail = [&](lbm_status st, const char* m) {
        if (err) *err = m;
        return st;
    };
    if (d.lattice != LBM_D2Q9_D2Q5 || !c->ck.flow || !c->ck.thermal || c->ck.bcx != 1 ||
        c->ck.bcy != 1 || c->ck.buoy || c->ck.tq != 5 ||
        d.batch != 1)
        return fail(LBM_E_UNSUPPORTED,
                    "the adjoint needs the channel lattice with flow, D2Q5 thermal, inlet/outlet, "
                    "walls on both sides, no buoyancy, batch 1");
    if (nsteps < 1 || K < 1) return fail(LBM_E_ARG, "nsteps and ckpt_every must be >= 1");
    RecLayout r{};
    r.state = align256((size_t)c->nplanes * c->P * c->esize);
    r.nseg = (nsteps + K - 1) / K;
    const int Kt = K < nsteps ? K : nsteps;
    r.tiles = chan_tiles(c->ck);
    size_t off = 0;
    r.offCk = off; off += (size_t)r.nseg * r.state;
    r.offTape = off; off += (size_t)(Kt + 1) * r.state;
    r.offLam = off; off += 2 * r.state;
    r.offDq = off; off += align256(4 * (size_t)d.nx * sizeof(double));
    r.offAcc = off; off += align256(2 * (size_t)r.tiles * sizeof(double));
    r.offGrad = off; off += align256(((size_t)d.nx + 2) * sizeof(double));
    r.total = off;
    *R = r;
    return LBM_OK;
}

template <typename S>
hipError_t chan_step_ptr(lbm_ctx* c, const S* a, S* b, long long t) {
    const double mod = 1.0 + c->flux_amp * std::sin(c->flux_omega * (double)t * c->dt);
    return launch_chan_step<S>(c->ck, a, b, aux_qw<S>(c), aux_uin<S>(c), aux_tin<S>(c), mod,
                               c->stream);
}

template <typename S>
hipError_t grad_impl(lbm_ctx* c, const RecLayout& R, double scale) {
    const int nx = c->desc.nx;
    char* w = c->rec_work;
    double* dq = (double*)(w + R.offDq);
    double* acc = (double*)(w + R.offAcc);
    double* grad = (double*)(w + R.offGrad);
    S* lam[2] = {(S*)(w + R.offLam), (S*)(w + R.offLam + R.state)};
    hipError_t e = hipMemsetAsync(dq, 0, 4 * (size_t)nx * sizeof(double), c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(acc, 0, 2 * (size_t)R.tiles * sizeof(double), c->stream);
    if (e != hipSuccess) return e;
    // seed from the final state (the context's current buffer)
    const long long tN = c->rec_t0 + c->rec_nsteps;
    const double modN = 1.0 + c->flux_amp * std::sin(c->flux_omega * (double)tN * c->dt);
    const S* fin = (const S*)bufA(c);
    e = launch_adj_seed<S>(c->ck, fin, aux_qw<S>(c), c->dx * c->rho_cp / c->dt * modN, modN, c->Dh,
                           c->k_cond, c->dx, c->rho_cp, c->cs2, c->rec_obj.x_dev, c->rec_obj.w_tout,
                           c->rec_obj.w_nu, lam[0], dq + 2 * nx, dq + 3 * nx, c->stream);
    if (e != hipSuccess) return e;
    int cur = 0;
    for (int sg = R.nseg - 1; sg >= 0; --sg) {
        const long long t0 = c->rec_t0 + (long long)sg * c->rec_K;
        const int len = (sg == R.nseg - 1) ? c->rec_nsteps - sg * c->rec_K : c->rec_K;
        S* tape = (S*)(w + R.offTape);
        e = hipMemcpyAsync(tape, w + R.offCk + (size_t)sg * R.state, R.state, hipMemcpyDeviceToDevice,
                           c->stream);
        if (e != hipSuccess) return e;
        for (int j = 0; j < len; ++j) {
            e = chan_step_ptr<S>(c, (const S*)((char*)tape + (size_t)j * R.state),
                                 (S*)((char*)tape + (size_t)(j + 1) * R.state), t0 + j);
            if (e != hipSuccess) return e;
        }
        for (int j = len - 1; j >= 0; --j) {
            const S* st = (const S*)((char*)tape + (size_t)j * R.state);
            const double mod = 1.0 + c->flux_amp * std::sin(c->flux_omega * (double)(t0 + j) * c->dt);
            e = launch_adj_step<S>(c->ck, c->ak, st, lam[cur], lam[cur ^ 1], mod, dq, dq + nx, acc,
                                   c->stream);
            if (e != hipSuccess) return e;
            cur ^= 1;
        }
    }
    return launch_adj_final(nx, R.tiles, scale, dq, dq + nx, dq + 2 * nx, dq + 3 * nx, acc, grad,
                            grad + nx, c->stream);
}

}  // namespace

extern "C" {

lbm_status lbm_query_record_bytes(const lbm_ctx* c, int nsteps, int ckpt_every, size_t* bytes) {
    if (!c || !bytes) return LBM_E_ARG;
    if (!c->has_params) return LBM_E_STATE;
    RecLayout R;
    lbm_status st = rec_layout(c, nsteps, ckpt_every, &R, nullptr);
    if (st != LBM_OK) return st;
    *bytes = R.total;
    return LBM_OK;
}

lbm_status lbm_record(lbm_ctx* c, int nsteps, int ckpt_every, const lbm_objective* obj, void* work,
                      size_t work_bytes, double* J) {
    if (!c) return LBM_E_ARG;
    if (!obj || !work || !J) return set_err(c, LBM_E_ARG, "obj, work and J are required");
    if (!c->has_state) return set_err(c, LBM_E_STATE, "no state");
    RecLayout R;
    lbm_status st = rec_layout(c, nsteps, ckpt_every, &R, &c->err);
    if (st != LBM_OK) return st;
    if (work_bytes < R.total || ((uintptr_t)work & 255) != 0)
        return set_err(c, LBM_E_ARG, "work buffer too small or not 256-byte aligned");
    if (obj->x_dev < 0 || obj->x_dev >= c->desc.nx) return set_err(c, LBM_E_ARG, "x_dev out of range");
    DeviceGuard g(c->device);
    char* w = (char*)work;
    c->has_record = false;
    const long long t0 = c->t;
    for (int sg = 0; sg < R.nseg; ++sg) {
        hipError_t e = hipMemcpyAsync(w + R.offCk + (size_t)sg * R.state, bufA(c),
                                      (size_t)c->nplanes * c->P * c->esize, hipMemcpyDeviceToDevice,
                                      c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "checkpoint copy");
        const int len = (sg == R.nseg - 1) ? nsteps - sg * ckpt_every : ckpt_every;
        st = lbm_step(c, len);
        if (st != LBM_OK) return st;
    }
    double nm = 0, tout = 0;
    st = lbm_nusselt(c, obj->x_dev, nullptr, nullptr, nullptr, &nm, &tout);
    if (st != LBM_OK) return st;
    *J = obj->w_tout * tout + obj->w_nu * nm;
    c->rec_work = w;
    c->rec_bytes = work_bytes;
    c->rec_nsteps = nsteps;
    c->rec_K = ckpt_every;
    c->rec_nseg = R.nseg;
    c->rec_t0 = t0;
    c->rec_obj = *obj;
    c->has_record = true;
    return LBM_OK;
}

lbm_status lbm_grad(lbm_ctx* c, double dL_dJ, double* dJ_dflux, double* dJ_dtau) {
    if (!c) return LBM_E_ARG;
    if (!dJ_dflux || !dJ_dtau) return set_err(c, LBM_E_ARG, "output arrays are required");
    if (!c->has_record) return set_err(c, LBM_E_STATE, "call lbm_record first");
    if (c->t != c->rec_t0 + c->rec_nsteps)
        return set_err(c, LBM_E_STATE, "the state moved since lbm_record");
    RecLayout R;
    lbm_status st = rec_layout(c, c->rec_nsteps, c->rec_K, &R, &c->err);
    if (st != LBM_OK) return st;
    DeviceGuard g(c->device);
    hipError_t e = c->desc.prec == LBM_FP64 ? grad_impl<double>(c, R, dL_dJ)
                                            : grad_impl<float>(c, R, dL_dJ);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint");
    const int nx = c->desc.nx;
    std::vector<double> h(nx + 2);
    e = hipMemcpyAsync(h.data(), c->rec_work + R.offGrad, h.size() * sizeof(double),
                       hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint");
    std::memcpy(dJ_dflux, h.data(), nx * sizeof(double));
    dJ_dtau[0] = h[nx];
    dJ_dtau[1] = h[nx + 1];
    return LBM_OK;
}

}  // extern "C"

extern "C" {

struct StateHeader {
    uint32_t magic, version;
    int32_t lattice, nx, ny, batch, prec, npop;
    uint64_t hash;
    int64_t t;
    uint64_t pop_bytes, phiu_bytes;
};

// State values between device and a host blob holding N values per plane:
// planes with stride P, or for a node-blocked state the node blocks with the
// padding of the last block left out (the full blocks in one copy, then the
// last block's N mod 64 nodes value by value).
static hipError_t copy_state(lbm_ctx* c, char* host, char* dev, bool to_host) {
    const size_t es = c->esize, row = (size_t)c->N * es;
    const hipMemcpyKind kind = to_host ? hipMemcpyDeviceToHost : hipMemcpyHostToDevice;
    if (!node_blocked(c->desc.lattice)) {
        const size_t pitch = (size_t)c->P * es;
        return to_host ? hipMemcpy2DAsync(host, row, dev, pitch, row, c->nplanes, kind, c->stream)
                       : hipMemcpy2DAsync(dev, pitch, host, row, row, c->nplanes, kind, c->stream);
    }
    const size_t blk = (size_t)kBlk * es, full = (size_t)(c->N / kBlk) * c->nplanes * blk;
    const size_t rest = (size_t)(c->N % kBlk) * es;
    hipError_t e = full ? (to_host ? hipMemcpyAsync(host, dev, full, kind, c->stream)
                                   : hipMemcpyAsync(dev, host, full, kind, c->stream))
                        : hipSuccess;
    if (e == hipSuccess && rest)
        e = to_host ? hipMemcpy2DAsync(host + full, rest, dev + full, blk, rest, c->nplanes, kind,
                                       c->stream)
                    : hipMemcpy2DAsync(dev + full, blk, host + full, rest, rest, c->nplanes, kind,
                                       c->stream);
    return e;
}

lbm_status lbm_save_state(lbm_ctx* c, void* host, size_t* bytes) {
    if (!c) return LBM_E_ARG;
    if (!bytes) return set_err(c, LBM_E_ARG, "bytes is NULL");
    // the blob holds the N node values of each plane, without the padding
    // between planes or after the last node block (which no kernel writes)
    const size_t row = (size_t)c->N * c->esize;
    const size_t pop = (size_t)c->nplanes * row;
    const size_t pu = 0;  // (phi u) is part of the state buffer
    const size_t need = sizeof(StateHeader) + pop + pu;
    if (!host) {
        *bytes = need;
        return LBM_OK;
    }
    if (*bytes < need) return set_err(c, LBM_E_ARG, "host buffer too small");
    if (!c->has_state) return set_err(c, LBM_E_STATE, "no state");
    DeviceGuard g(c->device);
    StateHeader hd{kMagic, kVersion, c->desc.lattice, c->desc.nx, c->desc.ny, c->desc.batch,
                   c->desc.prec, c->npop, c->hash, c->t, pop, pu};
    std::memcpy(host, &hd, sizeof hd);
    char* p = (char*)host + sizeof hd;
    hipError_t e = copy_state(c, p, bufA(c), true);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "save state");
    *bytes = need;
    return LBM_OK;
}

lbm_status lbm_load_state(lbm_ctx* c, const void* host, size_t bytes) {
    if (!c) return LBM_E_ARG;
    if (!host) return set_err(c, LBM_E_ARG, "host is NULL");
    if (!c->has_params) return set_err(c, LBM_E_STATE, "lbm_set_params_SI must come first");
    if (bytes < sizeof(StateHeader)) return set_err(c, LBM_E_STATE, "state blob truncated");
    StateHeader hd;
    std::memcpy(&hd, host, sizeof hd);
    const size_t row = (size_t)c->N * c->esize;
    const size_t pop = (size_t)c->nplanes * row;
    const size_t pu = 0;  // (phi u) is part of the state buffer
    if (hd.magic != kMagic || hd.version != kVersion) return set_err(c, LBM_E_STATE, "not a state blob");
    if (hd.lattice != c->desc.lattice || hd.nx != c->desc.nx || hd.ny != c->desc.ny ||
        hd.batch != c->desc.batch || hd.prec != c->desc.prec || hd.npop != c->npop ||
        hd.pop_bytes != pop || hd.phiu_bytes != pu)
        return set_err(c, LBM_E_STATE, "state blob is for another description");
    if (hd.hash != c->hash) return set_err(c, LBM_E_STATE, "state blob is for other parameters");
    if (bytes < sizeof hd + pop + pu) return set_err(c, LBM_E_STATE, "state blob truncated");
    DeviceGuard g(c->device);
    const char* p = (const char*)host + sizeof hd;
    c->cur = 0;
    hipError_t e = reset_persist(c);
    if (e == hipSuccess) e = reset_watch(c);
    if (e == hipSuccess) e = copy_state(c, const_cast<char*>(p), c->popA, false);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "load state");
    c->t = hd.t;
    c->has_state = true;
    return LBM_OK;
}

}  // extern "C"

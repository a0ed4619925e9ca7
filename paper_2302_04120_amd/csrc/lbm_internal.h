// Internal declarations of liblbm: context, kernel-argument structs and the
// launch wrappers the C-ABI layer calls.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "lbm.h"

namespace lbm {

// Node-block layout (every 2D and 3D lattice state): nodes in blocks of 64
// consecutive node indices, each block holding all npl values of its nodes,
// value by value (value i of node n at ((n / 64) npl + i) 64 + n mod 64).  A
// wave that loads 64 consecutive nodes reads one contiguous block of npl x
// 256 bytes (FP32); with one plane array per population the same wave opens
// npl separate streams.  Measured against planes: two-phase D2Q9 single step
// 2.25 -> 2.01 ms (67 M nodes), two-step launch 2.31 -> 2.25 ms, D3Q19 and 3D
// two-phase steps 3-7 % faster.  The padding of the last block is never read
// or written.
constexpr int kBlk = 64;
// the lattices whose state is stored in node blocks (the others keep one
// plane of stride P per population)
inline bool node_blocked(int lattice) {
    return lattice == LBM_D2Q9_PHASE || lattice == LBM_D2Q9_D2Q5 || lattice == LBM_D3Q19 ||
           lattice == LBM_D3Q19_PHASE;
}
__host__ __device__ __forceinline__ long long bidx(int npl, int i, long long n) {
    return ((n >> 6) * npl + i) * kBlk + (n & (kBlk - 1));
}

// Kernel constants of the D2Q9 momentum + D2Q5 temperature step.  Everything
// is pre-scaled by the host into lattice-normalised form (velocities in units
// of c, forces as F dt^2/dx, rates as Lambda dt): the dimensional matrix of
// Sec. 3 is the lattice matrix with rows scaled by c^order, so moment-space
// relaxation gives identical populations in either normalisation.
struct ChanK {
    int nx, ny, batch;
    long long P;          // plane stride of the FP64 staging fields (elements)
    int npl;              // values per node of the state (node blocks): f 9, then g 5 or 9
    int bcx, bcy;         // 0 periodic; bcx 1 inlet/outlet, 2 fixed-T walls;
                          // bcy 1 walls, 2 wall at y- + symmetry plane at y+
    int flow, thermal, flow_mrt, thermal_mrt;
    double rho_ref;
    double Lf[9];         // flow rates * dt in the order rho,e,eps,jx,qx,jy,qy,pxx,pxy
    double Ft[2];         // body force * dt^2 / dx
    int tq;               // thermal lattice: 5 (D2Q5) or 9 (D2Q9)
    double Lt[9];         // thermal rates * dt: D2Q5 T,jx,jy,e,pxx; D2Q9 the flow basis
    double qdt;           // qdot * dt (K)
    double c;             // lattice speed dx/dt (m/s), for outputs
    double T_ref;
    double Tw[2];         // bcx 2: wall temperature - T_ref at x- and x+ (K)
    int buoy;             // Boussinesq force on
    double Bt[2];         // its lattice force per kelvin: -rho_ref beta g dt^2 / dx
};

struct PhaseK {
    int nx, ny, batch;
    long long P;
    int bcy;              // 0 periodic, 1 walls (x periodic)
    int z_mrt, qy_printed, visc_mode;
    double rho_l, rho_g;
    double nuh_l, nuh_g;  // lattice viscosities nu dt/dx^2 (visc_mode 0)
    double zh_l, zh_g;    // zeta dt/dx^2 (visc_mode 1)
    double w_phi;         // dt / tau_phi
    double beta;          // 12 sigma / W        (Pa)
    double kap6;          // 6 kappa / dx^2      (Pa): mu = 4 beta phi(phi-1)(phi-1/2) - kap6 L
    double fs_scale;      // 3 dt^2 / dx^2: F~_s = mu G fs_scale
    double Fbt[2];        // body force * dt^2 / dx
    double dxW;           // dx / W
    double Geps;          // |G| threshold for n = 0 (= normal_eps dx / 3)
    double c, cs2;        // outputs
};

// Derivatives of the relaxation rates (times dt) with respect to tau and tau_T,
// in 1/s, and the flux boundary coefficient dt / (dx rho_cp).
struct AdjK {
    double dLf[9];
    double dLt[5];
    double qgrad;
};

// D3Q19 momentum: lattice-normalised like ChanK
struct D3K {
    int nx, ny, nz, batch;
    long long P;
    int bcx, bcy, bcz;    // per axis: 0 periodic, 1 halfway walls on both sides
    double rho_ref;
    double L[19];         // rates * dt in the basis order rho, e, eps, j_x, q_x, j_y, q_y,
                          // j_z, q_z, 3p_xx, 3pi_xx, p_ww, pi_ww, p_xy, p_yz, p_xz, m_x, m_y, m_z
    double Ft[3];         // body force * dt^2 / dx
    double c;             // dx / dt (outputs)
};

// 3D two-phase model (h_i and z_i on D3Q19), lattice-normalised like PhaseK
struct P3K {
    int nx, ny, nz, batch;
    long long P;
    int bcx, bcy, bcz;    // per axis: 0 periodic, 1 halfway walls on both sides
    int z_mrt, visc_mode;
    double rho_l, rho_g;
    double nuh_l, nuh_g;  // nu dt / dx^2 (visc_mode 0)
    double zh_l, zh_g;    // zeta dt / dx^2 (visc_mode 1)
    double w_phi;         // dt / tau_phi
    double beta;          // 12 sigma / W (Pa)
    double kap6;          // 6 kappa / dx^2 (Pa)
    double fs_scale;      // 3 dt^2 / dx^2
    double Fbt[3];        // body force * dt^2 / dx
    double dxW;           // dx / W
    double Geps;          // |G| threshold for n = 0
    double c, cs2;        // outputs
};

struct D1K {
    int n, q;
    double w_tau;         // dt / tau
    double qdt;           // qdot * dt
    double ufac;          // c u / c_s^2 (multiplies e_i in the equilibrium)
    double T0, TL;
};

}  // namespace lbm

struct lbm_ctx {
    lbm_desc desc;
    int device;
    hipStream_t stream;
    // layout
    long long N;          // nodes per replica * batch
    long long P;          // plane stride
    int npop;             // population planes (non-finite checks, reductions)
    int nplanes;          // planes per state buffer: npop, plus (phi u) for PHASE
    size_t esize;         // bytes per population value
    char* popA;
    char* popB;
    char* aux;            // flux (qw), inlet_u (uin), inlet_T (tin): storage type
    double* staging;      // 8 planes of FP64
    double* partial;      // reduction partials
    double* scratch;      // device address of the static scratch of lbm_reduce_noalloc
    unsigned long long* watch;  // first step with a non-finite state seen (~0: none)
    int watch_every = 4096;     // steps between non-finite checks (0: off)
    double fp32_forcing_share = 0.0;  // per-step share of the slowest forced mode (guard)
    double* small;        // small FP64 results
    int cur;              // 0: A holds the state, 1: B holds it
    long long t;          // steps since init
    bool has_params, has_state;
    lbm_params_si sp;     // SI scalars (array pointers cleared)
    lbm::ChanK ck;
    lbm::PhaseK pk;
    lbm::D1K dk;
    lbm::D3K d3k;
    lbm::P3K p3k;
    char* phi3;           // D3Q19_PHASE: phi of the current state (one plane, storage type)
    double flux_amp, flux_omega, dt;
    double k_cond, Dh, dx, rho_cp;
    std::string err;
    uint64_t hash;
    // adjoint
    lbm::AdjK ak;
    double cs2;
    bool has_record;
    char* rec_work;
    size_t rec_bytes;
    int rec_nsteps, rec_K, rec_nseg;
    long long rec_t0;
    lbm_objective rec_obj;
    // step replay: graph_steps (even) steps captured once per buffer parity
    // on a private stream and replayed on `stream`; 0 disables
    int graph_steps = 64;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t step_graph[2] = {nullptr, nullptr};
    int graph_swaps[2] = {0, 0};  // buffer swaps made by each captured graph
    // two-phase steps: 0 automatic, 1 single-step kernel only, 2 two-step
    // kernel whenever the grid allows it, 3 many steps per cooperative launch
    int fusion = 0;
    int tb2_seg = 0;                    // rows per two-step workgroup (0: kernel not usable)
    unsigned* persist_flags = nullptr;  // kPersistMaxTiles step counters, then the error word
    unsigned persist_epoch = 0;         // steps taken by persistent launches since the reset
};

namespace lbm {

constexpr int kRedBlocks = 256;  // first-pass blocks per replica and field

// launch wrappers (lbm_kernels.hip); all enqueue on s and return hipGetLastError()
// one channel step from state a to state b (node blocks: f 0-8, g from 9)
template <typename S>
hipError_t launch_chan_step(const ChanK& k, const S* a, S* b, const S* qw, const S* uin,
                            const S* tin, double mod, hipStream_t s);
// two channel steps in one launch from state a to state b; needs
// chan_tb2_fits.  mod0, mod1: the wall-flux modulations of the two steps;
// seg: rows per workgroup (chan_tb2_seg, fixed when the parameters are set)
bool chan_tb2_fits(const ChanK& k);
double chan_tb2_lane_use(const ChanK& k);
long long chan_tb2_workgroups(const ChanK& k, int seg);
template <typename S>
int chan_tb2_seg(const ChanK& k);
template <typename S>
hipError_t launch_chan_tb2(const ChanK& k, const S* a, S* b, const S* qw, const S* uin,
                           const S* tin, double mod0, double mod1, int seg, hipStream_t s);
// one two-phase step from state a to state b (node-block layout); arith64:
// evaluate the step in FP64 on FP32 storage (S = float)
template <typename S>
hipError_t launch_phase_step(const PhaseK& k, const S* a, S* b, bool arith64, hipStream_t s);
// two steps in one launch; the whole state (populations and (phi u)) moves
// from buffer a to buffer b; needs phase_tb2_fits.  seg: rows per workgroup
// (phase_tb2_seg, fixed when the parameters are set)
bool phase_tb2_fits(const PhaseK& k);
// whether rows go in x-tiles (nx not a multiple of 64 up to 256), and the
// share of the launched lanes whose columns are stored
bool phase_tb2_tiled(const PhaseK& k);
double phase_tb2_lane_use(const PhaseK& k);
template <typename S>
int phase_tb2_seg(const PhaseK& k);
long long phase_tb2_workgroups(const PhaseK& k, int seg);
template <typename S>
hipError_t launch_phase_tb2(const PhaseK& k, const S* a, S* b, int seg, hipStream_t s);
// *first = min(*first, t) if any node value of the nplanes planes is not
// finite (plane stride P, or the node-block layout when blocked)
template <typename S>
hipError_t launch_nonfinite_watch(const S* pops, long long P, long long N, int nplanes,
                                  bool blocked, unsigned long long t, unsigned long long* first,
                                  hipStream_t s);
// many steps in one cooperative launch for grids that split into at most
// kPersistMaxTiles tiles of 512 threads (phase_persist_fits); flags: one step
// counter per tile (zeroed with the state, advanced to epoch0 + steps), err:
// set when a bounded wait ran out
#ifndef LBM_PERSIST_MAX_TILES
#define LBM_PERSIST_MAX_TILES 16
#endif
constexpr int kPersistMaxTiles = LBM_PERSIST_MAX_TILES;
constexpr size_t kPersistFlagBytes = 256 * ((kPersistMaxTiles + 1) * 4 / 256 + 1);
bool phase_persist_fits(const PhaseK& k);
template <typename S>
hipError_t launch_phase_persist(const PhaseK& k, S* A, S* B, int nsteps, unsigned epoch0,
                                unsigned* flags, unsigned* err, bool arith64, hipStream_t s);
hipError_t launch_d1(const D1K& k, double* g, int nsteps, hipStream_t s);

template <typename S>
hipError_t launch_chan_init(const ChanK& k, const double* fields, S* a, hipStream_t s);
template <typename S>
hipError_t launch_phase_init(const PhaseK& k, const double* fields, S* a, hipStream_t s);
hipError_t launch_d1_init(const D1K& k, const double* T, double* g, hipStream_t s);

// D3Q19 (lbm_d3q19.hip)
long long d3_tiles(const D3K& k);
template <typename S>
hipError_t launch_d3_step(const D3K& k, const S* fc, S* fn, hipStream_t s);
template <typename S>
hipError_t launch_d3_init(const D3K& k, const double* fields, S* f, hipStream_t s);
template <typename S>
hipError_t launch_d3_macros(const D3K& k, const S* f, double* out, hipStream_t s);

// 3D two-phase (lbm_phase3d.hip).  A step is two launches: phi of the stored
// state into one plane, then the step kernel, which reads phi through an LDS
// tile with a one-node halo.  Buffer planes: h 0-18, z 19-37, the low part of
// h_0 at 38 (FP32 only), then (phi u) of the previous step (3 planes).
template <typename S>
hipError_t launch_p3_step(const P3K& k, const S* a, S* b, S* phi, hipStream_t s);
template <typename S>
hipError_t launch_p3_init(const P3K& k, const double* fields, S* a, hipStream_t s);
template <typename S>
hipError_t launch_p3_macros(const P3K& k, const S* a, S* phi, double* out, hipStream_t s);

// macros into staging slots [8][P]: rho, p, ux, uy, T, phi, mu, uz
template <typename S>
hipError_t launch_chan_macros(const ChanK& k, const S* a, double* out, hipStream_t s);
template <typename S>
hipError_t launch_phase_macros(const PhaseK& k, const S* a, double* out, hipStream_t s);
hipError_t launch_d1_macros(const D1K& k, const double* g, double* out, long long P,
                            hipStream_t s);

// per-replica FP64 sums: out[b*4 + f], f = mass, phase, energy, nonfinite
template <typename S>
hipError_t launch_reduce(int lattice, const ChanK& ck, const PhaseK& pk, const D1K& dk,
                         const D3K& d3, const P3K& p3, const S* pops, int npop, double* partial,
                         double* out, hipStream_t s);

// qsi converts the stored scaled flux to W/m^2 (including the time modulation);
// small receives (mean Nu over x >= x_dev, Tb[nx-1])
template <typename S>
hipError_t launch_nusselt(const ChanK& k, const S* a, const S* qw, double qsi, double Dh,
                          double kc, double dx, int x_dev, double* Tb, double* Tw, double* Nu,
                          double* small, hipStream_t s);

// ---- discrete adjoint of the heated channel (lbm_adjoint.hip)
// The adjoint state has the layout of the channel state (node blocks: lambda_f
// 0-8, lambda_g 9-13).  Seed at the final state st: lambda into l, and the
// objective's direct derivatives per column (dq_direct[x], dtauT_direct[x])
template <typename S>
hipError_t launch_adj_seed(const ChanK& k, const S* st, const S* qw, double qsi, double mod,
                           double Dh, double kc, double dx, double rho_cp, double cs2, int x_dev,
                           double w_tout, double w_nu, S* l, double* dq_direct,
                           double* dtauT_direct, hipStream_t s);
// one reverse step: lambda(n) into l from lambda(n+1) in ln and the state st at n
template <typename S>
hipError_t launch_adj_step(const ChanK& k, const AdjK& a, const S* st, const S* ln, S* l,
                           double mod, double* dq_bot, double* dq_top, double* dtau_acc,
                           hipStream_t s);
// gradient assembly (fixed order): grad_flux[nx], grad_tau[2]
hipError_t launch_adj_final(int nx, int ntiles, double scale, const double* dq_bot,
                            const double* dq_top, const double* dq_direct,
                            const double* dtauT_direct, const double* dtau_acc,
                            double* grad_flux, double* grad_tau, hipStream_t s);
int chan_tiles(const ChanK& k);

}  // namespace lbm

// lbfs_api.hip -- host side of the C ABI declared in include/lbfs.h.
//
// The solver state lives in one caller-owned device buffer, carved into 256-byte
// aligned segments: the instance descriptor, the tile lists, FP64 partials and
// results, and 18 SoA fields (W, W1, W2 of 5 fields each, phi' twice, S) with the row
// pitch padded to 64 elements. No device allocation happens inside the library.
#include "lbfs.h"
#include "lbfs_internal.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <map>
#include <mutex>
#include <new>
#include <vector>

using namespace lbfs;

namespace {

constexpr size_t ALIGN = 256;
constexpr int NFIELDS = 18;   // W[5], W1[5], W2[5], phi[0], S, phi[1]
// The order parameter C of W, W1 and W2 is stored in FP64 in both precisions: in FP64
// in fields 4, 9 and 14, in FP32 in three FP64 fields after the 18 (fields 4, 9 and 14
// are then unused, and stay in place so that fields 5-14 remain one scratch range).
constexpr int NCFIELDS = 3;
constexpr uint32_t CKPT_MAGIC = 0x5346424cu;   // "LBFS"

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int tiles_of(int n, int t) { return (n + t - 1) / t; }
int count_tiles(int nx, int ny, TileShape S) { return tiles_of(nx, S.tx) * tiles_of(ny, S.ty); }

// tiles of one instance (inst: its index in the descriptor array), row-major or, with
// `blocked`, in the order of tile_at; idx numbers them row-major inside the instance (the
// slot of its partial sums, which are reduced in that order). The magnetic kernels take
// the blocked order: their tiles are whole cache lines wide and their halo is deep. The
// stage tiles are not: a block edge inside a cache line makes two XCDs read and write
// parts of that line, which cost more than the halo saved (measured).
void append_tiles(std::vector<Tile>& out, int inst, int nx, int ny, TileShape S, bool blocked = false)
{
    const int ntx = tiles_of(nx, S.tx), nty = tiles_of(ny, S.ty);
    for (int k = 0; k < ntx * nty; k++) {
        int tx = k % ntx, ty = k / ntx;
        if (blocked) tile_at(k, ntx, nty, S.tx, S.ty, tx, ty);
        out.push_back(Tile{inst, tx * S.tx, ty * S.ty, ty * ntx + tx});
    }
}

// Segments of one instance's state. Tile lists and partial sums have room for the
// largest tile count of any candidate shape, so the tile shapes can change at run time.
struct Layout {
    int pitch = 0;
    size_t esize = 0, field_bytes = 0, cfield_bytes = 0;
    int cap_stage = 0, cap_mag = 0, tiles_pt_x = 0, tiles_pt_y = 0;
    size_t off_inst = 0, off_tstage = 0, off_tmag = 0, off_tpt = 0, off_part = 0, off_mpart = 0, off_res = 0,
           off_fields = 0, off_cfields = 0, total = 0;
    int ntile_pt() const { return tiles_pt_x * tiles_pt_y; }
};

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// the automatic Runge-Kutta step: half a cell of the streaming speed (dx / 2, the
// acoustic number cs dt / dx = 0.29) unless a diffusivity needs less (0.4 dx^2 / D_max,
// D the kinematic viscosity and thermal diffusivity of every phase)
double auto_dt(const lbfs_params& p)
{
    double dmax = 0.0;
    for (int k = 0; k < 3; k++) {
        dmax = std::fmax(dmax, p.mu[k] / p.rho[k]);
        dmax = std::fmax(dmax, p.lambda[k] / (p.rho[k] * p.cp[k]));
    }
    const double dtd = dmax > 0.0 ? 0.4 * p.dx * p.dx / dmax : 0.5 * p.dx;
    return std::fmin(0.5 * p.dx, dtd);
}

int validate(const lbfs_params* p)
{
    if (!p) return LBFS_E_INVAL;
    if (p->abi_version != LBFS_ABI_VERSION) return LBFS_E_ABI;
    if (p->nx < 4 || p->ny < 4 || p->nx > (1 << 20) || p->ny > (1 << 20)) return LBFS_E_INVAL;
    // at most 2^30 cells: every cell, face and padded-row index of the kernels then fits
    // a 32-bit int
    if ((int64_t)p->nx * p->ny > ((int64_t)1 << 30)) return LBFS_E_INVAL;
    if (p->precision != LBFS_FP32 && p->precision != LBFS_FP64) return LBFS_E_INVAL;
    if (!finite_pos(p->dx) || !(p->dt == 0.0 || finite_pos(p->dt))) return LBFS_E_INVAL;   // 0: automatic
    if (p->dt_stream != 0.0 && std::fabs(p->dt_stream - 0.5 * p->dx) > 1e-12 * p->dx) return LBFS_E_INVAL;
    for (int k = 0; k < 3; k++) {
        if (!finite_pos(p->rho[k]) || !finite_pos(p->mu[k]) || !finite_pos(p->cp[k]) ||
            !finite_pos(p->lambda[k]))
            return LBFS_E_INVAL;
        if (!std::isfinite(p->chi[k]) || p->chi[k] <= -1.0) return LBFS_E_INVAL;
    }
    if (!std::isfinite(p->latent) || p->latent < 0.0) return LBFS_E_INVAL;
    if (!std::isfinite(p->t_melt) || !std::isfinite(p->t_init)) return LBFS_E_INVAL;
    if (!std::isfinite(p->t_liquidus) || p->t_liquidus < p->t_melt) return LBFS_E_INVAL;
    if (!finite_pos(p->mu0) || !std::isfinite(p->h0) || p->h0 < 0.0) return LBFS_E_INVAL;
    if (!std::isfinite(p->field_angle_deg) || !std::isfinite(p->gravity[0]) || !std::isfinite(p->gravity[1]))
        return LBFS_E_INVAL;
    if (!std::isfinite(p->sigma) || p->sigma < 0.0 || !finite_pos(p->xi)) return LBFS_E_INVAL;
    if (!std::isfinite(p->mobility) || p->mobility < 0.0) return LBFS_E_INVAL;
    if (!std::isfinite(p->tau_g) || p->tau_g <= 0.5) return LBFS_E_INVAL;
    if (!std::isfinite(p->drop_cx) || !std::isfinite(p->drop_cy) || !std::isfinite(p->drop_radius))
        return LBFS_E_INVAL;
    if (p->init_kind != LBFS_INIT_DROPLET && p->init_kind != LBFS_INIT_UNIFORM) return LBFS_E_INVAL;
    if (!std::isfinite(p->c_init)) return LBFS_E_INVAL;
    for (int a = 0; a < 2; a++)
        if (p->periodic[a] != 0 && p->periodic[a] != 1) return LBFS_E_INVAL;
    for (int w = 0; w < 4; w++) {
        if (p->thermal_bc[w] != LBFS_TBC_ADIABATIC && p->thermal_bc[w] != LBFS_TBC_FIXED) return LBFS_E_INVAL;
        if (p->mag_bc[w] != LBFS_MBC_INSULATING && p->mag_bc[w] != LBFS_MBC_FIXED) return LBFS_E_INVAL;
        if (!std::isfinite(p->thermal_val[w])) return LBFS_E_INVAL;
        if (!(p->contact_angle_deg[w] > 0.0 && p->contact_angle_deg[w] < 180.0)) return LBFS_E_INVAL;
    }
    if (p->sweeps < 0 || p->sweeps > 1000) return LBFS_E_INVAL;
    if (!(p->sor_omega > 0.0 && p->sor_omega < 2.0)) return LBFS_E_INVAL;
    if (p->mag_method != LBFS_MAG_SWEEPS && p->mag_method != LBFS_MAG_LBFS && p->mag_method != LBFS_MAG_MULTIGRID)
        return LBFS_E_INVAL;
    // multigrid: walls on every side, a fixed number of cycles per step
    if (p->mag_method == LBFS_MAG_MULTIGRID && (p->periodic[0] || p->periodic[1] || p->mag_max_iters != 0))
        return LBFS_E_INVAL;
    if (!finite_pos(p->mag_lbfs_d) || !std::isfinite(p->mag_lbfs_dtau) || p->mag_lbfs_dtau < 0.0)
        return LBFS_E_INVAL;
    if (p->mag_max_iters < 0 || p->mag_max_iters > 100000) return LBFS_E_INVAL;
    if (p->mag_max_iters > 0 && (p->sweeps < 1 || !std::isfinite(p->mag_tol) || p->mag_tol < 0.0))
        return LBFS_E_INVAL;
    if (!std::isfinite(p->init_omega) || p->init_omega >= 2.0) return LBFS_E_INVAL;
    if (!std::isfinite(p->init_tol) || p->init_tol < 0.0 || p->init_max < 0 || p->init_check < 0)
        return LBFS_E_INVAL;
    // a red-black colouring of a periodic axis needs an even number of cells
    if ((p->periodic[0] && (p->nx & 1)) || (p->periodic[1] && (p->ny & 1))) return LBFS_E_INVAL;
    // the applied-field potential is not periodic along an axis the field crosses
    const double th = p->field_angle_deg * M_PI / 180.0;
    const double hx = p->h0 * std::cos(th), hy = p->h0 * std::sin(th);
    if (p->periodic[0] && std::fabs(hx) > 1e-12 * p->h0) return LBFS_E_INVAL;
    if (p->periodic[1] && std::fabs(hy) > 1e-12 * p->h0) return LBFS_E_INVAL;
    // explicit stability of the diffusive and acoustic parts
    double dmax = 0.0;
    for (int k = 0; k < 3; k++) {
        dmax = std::fmax(dmax, p->mu[k] / p->rho[k]);
        dmax = std::fmax(dmax, p->lambda[k] / (p->rho[k] * p->cp[k]));
    }
    if (dmax * p->dt / (p->dx * p->dx) > 0.5) return LBFS_E_INVAL;   // (an automatic step is within)
    if (std::sqrt(1.0 / 3.0) * p->dt / p->dx > 1.0) return LBFS_E_INVAL;
    return LBFS_OK;
}

// the magnetic tile shape a step over `cells` cells takes unless shapes are given
// (measured per step: 32 x 8 fastest on 128^2 and 256^2, 64 x 16 on 512^2 by 9%, 64 x 32
// on 1024^2: a larger tile recomputes fewer halo cells once the tiles fill the GPU)
int default_mag_shape(size_t cells)
{
    return cells > (size_t)512 * 512 ? 1 : (cells > ((size_t)1 << 17) ? 2 : 0);
}

// the stage tile shape a step over `cells` cells takes unless shapes are given: the
// table's first, except in FP64 above 512^2, where 12 x 7 tiles (84 cells, still four
// workgroups per CU) do fewer halo cells and idle face lanes per cell (measured per
// step: 257.8 against 264.5 us for 10 x 8 on 1024^2, 1047.9 against 1078.2 on 2048^2;
// 10 x 8 stays ahead on 256^2 and below)
constexpr int F64_LARGE_STAGE_SHAPE = 4;
static_assert(STAGE_SHAPES_F64[F64_LARGE_STAGE_SHAPE].tx == 12 && STAGE_SHAPES_F64[F64_LARGE_STAGE_SHAPE].ty == 7,
              "the FP64 large-grid stage shape is 12 x 7");
int default_stage_shape(bool f64, size_t cells)
{
    return f64 && cells > (size_t)512 * 512 ? F64_LARGE_STAGE_SHAPE : 0;
}

Layout make_layout(const lbfs_params* p)
{
    Layout L;
    L.esize = p->precision == LBFS_FP64 ? 8 : 4;
    L.pitch = (int)align_up((size_t)p->nx, 64);
    L.field_bytes = align_up((size_t)L.pitch * p->ny * L.esize, ALIGN);
    for (int k = 0; k < NSTAGE_SHAPES; k++) {
        const int n = count_tiles(p->nx, p->ny, stage_shape(p->precision == LBFS_FP64, k));
        L.cap_stage = n > L.cap_stage ? n : L.cap_stage;
    }
    for (int k = 0; k < NMAG_SHAPES; k++) {
        const int n = count_tiles(p->nx, p->ny, MAG_SHAPES[k]);
        L.cap_mag = n > L.cap_mag ? n : L.cap_mag;
    }
    L.tiles_pt_x = tiles_of(p->nx, PT_TX);
    L.tiles_pt_y = tiles_of(p->ny, PT_TY);
    size_t off = 0;
    L.off_inst = off; off = align_up(off + sizeof(DevInst), ALIGN);
    L.off_tstage = off; off = align_up(off + sizeof(Tile) * L.cap_stage, ALIGN);
    L.off_tmag = off; off = align_up(off + sizeof(Tile) * L.cap_mag, ALIGN);
    L.off_tpt = off; off = align_up(off + sizeof(Tile) * L.ntile_pt(), ALIGN);
    L.off_part = off; off = align_up(off + sizeof(double) * NPART * L.cap_stage, ALIGN);
    // residual partials (per magnetic tile, or per stage tile when stage 1 runs the
    // sweeps) and the convergence flag
    L.off_mpart = off; off = align_up(off + sizeof(double) * (std::max(L.cap_mag, L.cap_stage) + 1), ALIGN);
    L.off_res = off; off = align_up(off + sizeof(double) * NRES, ALIGN);
    L.off_fields = off; off += L.field_bytes * NFIELDS;
    L.off_cfields = off;
    if (p->precision != LBFS_FP64) {
        L.cfield_bytes = align_up((size_t)L.pitch * p->ny * sizeof(double), ALIGN);
        off += L.cfield_bytes * NCFIELDS;
    } else {
        // the three fields stage 1 leaves for stages 2 and 3 (in FP32 they take the unused
        // FP32 slots of the order parameter)
        off += L.field_bytes * 3;
    }
    L.total = off + ALIGN;   // room to align the caller's base pointer
    return L;
}

// Geometric multigrid of one instance's magnetic system: level sizes and the element
// offsets of each level's arrays in a scratch region (the stage fields, free between
// steps). Level 0 solves for the potential itself (in its double buffer); its permeability
// is staged in its right-hand-side array while the face weights are formed.
struct MgCtx {
    int L = 0;                                   // levels; L - 1 is the coarsest
    int nx[24] = {}, ny[24] = {};
    size_t u[24] = {}, f[24] = {}, wx[24] = {}, wy[24] = {};
    char* scratch = nullptr;                     // base of the offsets
    void* phi[2] = {nullptr, nullptr};           // level-0 unknown, by potential parity
    int pitch = 0;                               // of the level-0 unknown
    int fixed_walls = 0;                         // bit w: wall w (W, E, S, N) holds the potential
    // per level, in level-0 cells: the cell width and the widths of the last column and
    // row (narrower where a halving had an odd count)
    int w[24] = {}, lastx[24] = {}, lasty[24] = {};
    // launch argument of the coarsening and prolongation between levels l and l + 1
    void geom(int l, int* g) const
    {
        g[0] = w[l];
        g[1] = lastx[l];
        g[2] = lasty[l];
        g[3] = lastx[l + 1];
        g[4] = lasty[l + 1];
    }
};

// V(2,2) cycles with the coarsest level by red-black SOR in one workgroup
constexpr int MG_PRE = 2, MG_POST = 2, MG_COARSE_SWEEPS = 40;

// The launches of one time step over a set of tile lists (one instance for a solver,
// the concatenated tiles of every live instance for a batch), with the potential
// buffer parity and the captured graphs of one step per parity.
struct Exec {
    bool f64 = false;
    int stage_shape = 0, mag_shape = 0;   // indices into the tile-shape tables
    int sweeps = 4;                      // sweeps, or pseudo-steps of the LBFS solve, per step
    double omega = 1.0;
    int mag_method = LBFS_MAG_SWEEPS;
    int mag_chunks = 1;                  // chunks of `sweeps` per step (convergence control)
    bool fused = false;                  // the sweeps run inside stage 1 (no magnetic launch)
    const MgCtx* mg = nullptr;           // multigrid plan (solvers whose method is multigrid)
    bool mres_stage = false;             // the last residual partials are per stage tile
    hipStream_t stream = nullptr;
    const DevInst* dinst = nullptr;
    int ninst = 0;
    const Tile* tiles_stage = nullptr;
    int nstage = 0;
    const Tile* tiles_mag = nullptr;
    int nmag = 0;
    int phase = 0;                       // potential buffer holding the current phi'
    // kf[0] of every instance holds the permeability of its current state (left there by
    // stage 3 of the last step, and no write of the state since)
    bool mu_ready = false;
    bool use_graph = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;   // timing of the next launch (profiled steps)
    int graph_steps = 1;                 // steps per replay of the longest graph
    // graph[li][ph]: glen[li] consecutive steps from potential buffer ph; the lengths are
    // the powers of two below graph_steps, then graph_steps itself
    static constexpr int NGLEN = 8;
    int glen[NGLEN] = {1};
    int nglen = 1;
    hipGraph_t graph[NGLEN][2] = {};
    hipGraphExec_t graph_exec[NGLEN][2] = {};
    // timing events of the profiled steps, created ahead (lbfs_prepare) or on first need
    // and kept, so that a profiled run creates none while the device waits
    std::vector<hipEvent_t> evpool;
    // the profiled run enqueued and not yet read: kernel kind of each timed launch
    bool prof_pending = false;
    std::vector<int> prof_kind;
    size_t prof_slots = 0;
};

// at least n events in the pool
hipError_t exec_events(Exec& E, size_t n)
{
    while (E.evpool.size() < n) {
        hipEvent_t e = nullptr;
        const hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        E.evpool.push_back(e);
    }
    return hipSuccess;
}

void exec_set_graph_steps(Exec& E, int gs)
{
    E.graph_steps = gs;
    E.nglen = 0;
    for (int l = 1; l < gs && E.nglen < Exec::NGLEN - 1; l *= 2) E.glen[E.nglen++] = l;
    E.glen[E.nglen++] = gs;
}

hipError_t exec_mag(Exec& E, int nsweeps, double omega, int residual)
{
    E.mres_stage = false;
    const int mi = E.mu_ready ? 1 : 0;
    return E.f64 ? launch_mag<double>(E.mag_shape, nsweeps, omega, residual, mi, &E.phase, E.dinst, E.tiles_mag,
                                      E.nmag, E.stream, E.ev0, E.ev1)
                 : launch_mag<float>(E.mag_shape, nsweeps, omega, residual, mi, &E.phase, E.dinst, E.tiles_mag,
                                     E.nmag, E.stream, E.ev0, E.ev1);
}

hipError_t exec_mag_lbfs(Exec& E, int nsteps, int residual, hipEvent_t e0, hipEvent_t e1, int gate)
{
    E.mres_stage = false;
    return E.f64 ? launch_mag_lbfs<double>(E.mag_shape, nsteps, residual, &E.phase, E.dinst, E.tiles_mag, E.nmag,
                                           E.stream, e0, e1, gate)
                 : launch_mag_lbfs<float>(E.mag_shape, nsteps, residual, &E.phase, E.dinst, E.tiles_mag, E.nmag,
                                          E.stream, e0, e1, gate);
}

hipError_t exec_mag_lbfs(Exec& E, int nsteps, int residual) { return exec_mag_lbfs(E, nsteps, residual, E.ev0, E.ev1, 0); }

template <typename T>
hipError_t mg_run(const Exec& E, const MgCtx& M, int ncycles, hipEvent_t e0)
{
    T* B = reinterpret_cast<T*>(M.scratch);
    T* u0 = static_cast<T*>(M.phi[E.phase]);
    auto U = [&](int l) { return l == 0 ? u0 : B + M.u[l]; };
    auto P = [&](int l) { return l == 0 ? M.pitch : M.nx[l]; };
    hipError_t e = launch_mg_setup0<T>(E.dinst, M.nx[0], M.ny[0], B + M.f[0], B + M.wx[0], B + M.wy[0], B + M.f[0],
                                       E.stream, e0);
    int g[5];
    for (int l = 0; l + 1 < M.L && e == hipSuccess; l++) {
        M.geom(l, g);
        e = launch_mg_coarsen<T>(M.nx[l], M.ny[l], B + M.wx[l], B + M.wy[l], M.nx[l + 1], M.ny[l + 1],
                                 B + M.wx[l + 1], B + M.wy[l + 1], g, E.stream);
    }
    const int c = M.L - 1;
    const int nmax = std::max(M.nx[c], M.ny[c]);
    const double om = 2.0 / (1.0 + std::sin(M_PI / std::max(nmax, 2)));
    for (int k = 0; k < ncycles && e == hipSuccess; k++) {
        for (int l = 0; l < c && e == hipSuccess; l++) {
            e = launch_mg_smooth<T>(M.nx[l], M.ny[l], P(l), U(l), B + M.f[l], B + M.wx[l], B + M.wy[l], MG_PRE,
                                    E.stream);
            if (e == hipSuccess)
                e = launch_mg_restrict<T>(M.nx[l], M.ny[l], P(l), U(l), B + M.f[l], B + M.wx[l], B + M.wy[l],
                                          M.nx[l + 1], M.ny[l + 1], B + M.f[l + 1], B + M.u[l + 1], E.stream);
        }
        if (e == hipSuccess)
            e = launch_mg_coarsest<T>(M.nx[c], M.ny[c], P(c), U(c), B + M.f[c], B + M.wx[c], B + M.wy[c],
                                      MG_COARSE_SWEEPS, om, E.stream);
        for (int l = c - 1; l >= 0 && e == hipSuccess; l--) {
            M.geom(l, g);
            e = launch_mg_prolong<T>(M.nx[l], M.ny[l], P(l), U(l), M.nx[l + 1], M.ny[l + 1], U(l + 1),
                                     M.fixed_walls, g, E.stream);
            if (e == hipSuccess)
                e = launch_mg_smooth<T>(M.nx[l], M.ny[l], P(l), U(l), B + M.f[l], B + M.wx[l], B + M.wy[l], MG_POST,
                                        E.stream);
        }
    }
    return e;
}

// ncycles multigrid cycles on the current potential (in place), then the residual
// partials by a sweep-free magnetic launch (which flips the potential buffer); the
// timing events bracket the first and the last launch
hipError_t exec_mg(Exec& E, int ncycles, int residual)
{
    if (!E.mg) return hipErrorInvalidValue;
    const hipEvent_t e0 = E.ev0;
    hipError_t e = E.f64 ? mg_run<double>(E, *E.mg, ncycles, e0) : mg_run<float>(E, *E.mg, ncycles, e0);
    if (e == hipSuccess && residual) {
        E.ev0 = nullptr;
        e = exec_mag(E, 0, 1.0, 1);
        E.ev0 = e0;
    }
    return e;
}

// The magnetic phase of a time step, by the instance's method, with the residual. With
// convergence control it is mag_chunks chunks of `sweeps` iterations; after the first,
// each chunk is gated by the convergence flag of the chunk before it, so a converged
// instance only copies its potential (the launch count, and with it the buffer flips,
// stays fixed and the step can be captured in a graph). The timing events bracket the
// whole phase.
// the magnetic phase of one step; `resid`: also the FP64 residual partials of its last
// launch, which lbfs_observe reduces (the convergence control needs them after every
// chunk, and multigrid writes them anyway)
hipError_t exec_mag_step(Exec& E, bool resid)
{
    hipError_t e = hipSuccess;
    E.mres_stage = false;
    const int r = (resid || E.mag_chunks > 1) ? 1 : 0;
    if (E.mag_method == LBFS_MAG_MULTIGRID) return exec_mg(E, E.sweeps, 1);
    for (int c = 0; c < E.mag_chunks && e == hipSuccess; c++) {
        const hipEvent_t a = c == 0 ? E.ev0 : nullptr, b = c == E.mag_chunks - 1 ? E.ev1 : nullptr;
        const int gate = c > 0;
        if (gate) e = launch_mag_gate(E.dinst, E.ninst, E.stream);
        if (e != hipSuccess) break;
        if (E.mag_method == LBFS_MAG_LBFS) {
            e = exec_mag_lbfs(E, E.sweeps, r, a, b, gate);
        } else {
            const int mi = E.mu_ready ? 1 : 0;
            e = E.f64 ? launch_mag<double>(E.mag_shape, E.sweeps, E.omega, r, mi, &E.phase, E.dinst, E.tiles_mag,
                                           E.nmag, E.stream, a, b, gate)
                      : launch_mag<float>(E.mag_shape, E.sweeps, E.omega, r, mi, &E.phase, E.dinst, E.tiles_mag,
                                          E.nmag, E.stream, a, b, gate);
        }
    }
    return e;
}

hipError_t exec_stage(Exec& E, int stage)
{
    return E.f64 ? launch_stage<double>(E.stage_shape, stage, E.phase, E.dinst, E.tiles_stage, E.nstage, E.stream,
                                        E.ev0, E.ev1)
                 : launch_stage<float>(E.stage_shape, stage, E.phase, E.dinst, E.tiles_stage, E.nstage, E.stream,
                                       E.ev0, E.ev1);
}

hipError_t exec_state_partials(Exec& E)
{
    return E.f64 ? launch_state_partials<double>(E.stage_shape, E.dinst, E.tiles_stage, E.nstage, E.stream)
                 : launch_state_partials<float>(E.stage_shape, E.dinst, E.tiles_stage, E.nstage, E.stream);
}

// stage 1 with the step's sweeps in front of it; flips the potential buffer
hipError_t exec_stage_fused(Exec& E)
{
    const hipError_t e =
        E.f64 ? launch_stage_fused<double>(E.stage_shape, E.phase, E.sweeps, E.omega, E.dinst, E.tiles_stage, E.nstage,
                                           E.stream, E.ev0, E.ev1)
              : launch_stage_fused<float>(E.stage_shape, E.phase, E.sweeps, E.omega, E.dinst, E.tiles_stage, E.nstage,
                                          E.stream, E.ev0, E.ev1);
    if (e == hipSuccess && E.nstage > 0) E.phase ^= 1;
    E.mres_stage = true;
    return e;
}

// one time step: magnetic phase and three Runge-Kutta stages, or the fused stage 1
// and stages 2 and 3 (the observables of the state are summed when they are read)
hipError_t exec_enqueue_step(Exec& E, bool resid = true)
{
    hipError_t e = E.fused ? exec_stage_fused(E) : exec_mag_step(E, resid);
    for (int st = E.fused ? 2 : 1; st <= 3 && e == hipSuccess; st++) e = exec_stage(E, st);
    if (e == hipSuccess) E.mu_ready = true;   // (stage 3 left the permeability in kf[0])
    return e;
}

void exec_drop_graphs(Exec& E)
{
    for (int l = 0; l < Exec::NGLEN; l++)
        for (int k = 0; k < 2; k++) {
            if (E.graph_exec[l][k]) (void)hipGraphExecDestroy(E.graph_exec[l][k]);
            if (E.graph[l][k]) (void)hipGraphDestroy(E.graph[l][k]);
            E.graph_exec[l][k] = nullptr;
            E.graph[l][k] = nullptr;
        }
}

void exec_release(Exec& E)
{
    exec_drop_graphs(E);
    for (hipEvent_t e : E.evpool) (void)hipEventDestroy(e);
    E.evpool.clear();
}

// capture glen[li] consecutive time steps starting from potential buffer `ph` into a HIP
// graph, once per length and buffer. A replay of a longer graph costs one launch for all
// its steps: the per-replay overhead of a graph launch is several microseconds, as much
// as a graph gap between kernels.
hipError_t exec_ensure_graph(Exec& E, int li, int ph)
{
    if (E.graph_exec[li][ph]) return hipSuccess;
    const int saved = E.phase;
    const bool saved_mres = E.mres_stage, saved_mu = E.mu_ready;
    E.phase = ph;
    // (a replay always follows a step: exec_run_steps runs one directly while the
    // permeability is not in kf[0])
    E.mu_ready = true;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(E.stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
        E.phase = saved;
        return e;
    }
    const int n = E.glen[li];
    // (the magnetic residual in the last step only: a replay ends every run of steps
    // that lbfs_observe can follow)
    for (int k = 0; k < n && e == hipSuccess; k++) e = exec_enqueue_step(E, k == n - 1);
    const hipError_t ec = hipStreamEndCapture(E.stream, &g);
    E.phase = saved;
    E.mres_stage = saved_mres;
    E.mu_ready = saved_mu;
    if (e == hipSuccess) e = ec;
    if (e == hipSuccess) e = hipGraphInstantiate(&E.graph_exec[li][ph], g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        E.graph_exec[li][ph] = nullptr;
        return e;
    }
    E.graph[li][ph] = g;
    return hipSuccess;
}

// steps per replay of the multi-step graph: 16, or LBFS_GRAPH_STEPS (1..64) from the
// environment (1: every replay is one step)
int graph_steps_setting()
{
    const char* v = std::getenv("LBFS_GRAPH_STEPS");
    if (!v || !*v) return 16;
    const long k = std::strtol(v, nullptr, 10);
    return k < 1 ? 1 : (k > 64 ? 64 : (int)k);
}

// potential-buffer flips of one step (one per magnetic launch)
int exec_step_flips(const Exec& E)
{
    if (E.fused || E.mag_method == LBFS_MAG_MULTIGRID) return 1;   // (the residual launch)
    const int kmax = E.mag_method == LBFS_MAG_LBFS ? RK_KMAX : MAG_KMAX;
    const int launches = E.sweeps == 0 ? 1 : (E.sweeps + kmax - 1) / kmax;
    return (launches * E.mag_chunks) & 1;
}

// up to `nmax` (>= 1) steps as one replay of the longest graph that many steps fill, or
// one step by direct launches where no graph of two or more steps fits (or graphs are
// off): a one-step graph replay costs a few microseconds more than the same kernels
// launched directly. The magnetic residual is written by the last step of a replay and
// by a direct step that is the last one asked for (nmax == 1), so the last step of any
// run leaves it. Returns the steps enqueued, 0 on a HIP error.
int exec_run_steps(Exec& E, int nmax)
{
    int li = 0;
    if (E.use_graph)
        while (li + 1 < E.nglen && E.glen[li + 1] <= nmax) li++;
    if (!E.use_graph || E.glen[li] < 2 || !E.mu_ready) return exec_enqueue_step(E, nmax == 1) == hipSuccess ? 1 : 0;
    const int n = E.glen[li];
    const int ph = E.phase;
    if (exec_ensure_graph(E, li, ph) != hipSuccess) return 0;
    if (hipGraphLaunch(E.graph_exec[li][ph], E.stream) != hipSuccess) return 0;
    E.phase = ph ^ ((n * exec_step_flips(E)) & 1);
    E.mres_stage = E.fused;
    return n;
}

// the timing events of profiled runs sampling up to this many steps are made ahead
constexpr int PREPARED_SAMPLES = 16;
constexpr int EVENTS_PER_SAMPLE = 8;   // start and end of the four kernel phases

// capture every graph exec_run_steps can replay (every length, from either potential
// buffer) without running it, and create the timing events of a profiled run
hipError_t exec_prepare(Exec& E)
{
    const hipError_t ee = exec_events(E, (size_t)PREPARED_SAMPLES * EVENTS_PER_SAMPLE);
    if (ee != hipSuccess) return ee;
    if (!E.use_graph || E.ninst == 0) return hipSuccess;
    for (int li = 0; li < E.nglen; li++)
        for (int ph = 0; ph < 2 && E.glen[li] >= 2; ph++) {
            const hipError_t e = exec_ensure_graph(E, li, ph);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

// Enqueue nsteps steps with HIP events around the kernel phases of every
// sample_every-th step; after_step() runs on the host after each enqueued step. The
// timings are read by exec_profiled_result (one profiled run pending at a time).
template <typename F>
int exec_profiled_start(Exec& E, int nsteps, int sample_every, F&& after_step)
{
    if (E.prof_pending) return LBFS_E_STATE;
    const int nsample = (nsteps + sample_every - 1) / sample_every;
    if (nsample > 4096) return LBFS_E_INVAL;
    const int per_step = EVENTS_PER_SAMPLE / 2;
    if (exec_events(E, (size_t)nsample * EVENTS_PER_SAMPLE) != hipSuccess) return LBFS_E_DEVICE;
    const std::vector<hipEvent_t>& ev = E.evpool;
    E.prof_kind.assign((size_t)nsample * per_step, 0);
    int rc = LBFS_OK;
    size_t slot = 0;
    // the launch itself timestamps the kernel's start and end into the events
    auto timed = [&](int k, auto&& launch) -> hipError_t {
        E.prof_kind[slot] = k;
        E.ev0 = ev[2 * slot];
        E.ev1 = ev[2 * slot + 1];
        const hipError_t e = launch();
        E.ev0 = E.ev1 = nullptr;
        slot++;
        return e;
    };
    for (int n = 0; n < nsteps && rc == LBFS_OK;) {
        if (n % sample_every == 0) {
            hipError_t e;
            if (E.fused) e = timed(LBFS_K_STAGE1, [&] { return exec_stage_fused(E); });
            else e = timed(LBFS_K_MAG, [&] { return exec_mag_step(E, n == nsteps - 1); });
            for (int st = E.fused ? 2 : 1; st <= 3 && e == hipSuccess; st++)
                e = timed(LBFS_K_STAGE1 + st - 1, [&] { return exec_stage(E, st); });
            if (e != hipSuccess) rc = LBFS_E_DEVICE;
            else E.mu_ready = true;
            after_step();
            n++;
            continue;
        }
        // the plain steps up to the next sampled one
        const int next = std::min(nsteps, (n / sample_every + 1) * sample_every);
        const int k = exec_run_steps(E, next - n);
        if (k == 0) rc = LBFS_E_DEVICE;
        for (int q = 0; q < k; q++) after_step();
        n += k;
    }
    E.prof_slots = slot;
    E.prof_pending = rc == LBFS_OK;
    return rc;
}

// wait for the pending profiled run and average its timed launches per kernel kind
int exec_profiled_result(Exec& E, double* kernel_ms, int32_t* launches)
{
    if (!E.prof_pending) return LBFS_E_STATE;
    E.prof_pending = false;
    int rc = hipStreamSynchronize(E.stream) == hipSuccess ? LBFS_OK : LBFS_E_DEVICE;
    for (int k = 0; k < LBFS_NKERNELS; k++) {
        kernel_ms[k] = 0.0;
        launches[k] = 0;
    }
    if (rc == LBFS_OK)
        for (size_t q = 0; q < E.prof_slots; q++) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, E.evpool[2 * q], E.evpool[2 * q + 1]) != hipSuccess) {
                rc = LBFS_E_DEVICE;
                break;
            }
            kernel_ms[E.prof_kind[q]] += ms;
            launches[E.prof_kind[q]] += 1;
        }
    for (int k = 0; k < LBFS_NKERNELS; k++)
        if (launches[k] > 0) kernel_ms[k] /= launches[k];
    return rc;
}

// the descriptor's parameters in one precision, with the kernels' derived constants
template <typename T>
void fill_coef(Coef<T>& K, const DevInst& I)
{
    for (int k = 0; k < 3; k++) {
        K.rho[k] = T(I.rho[k]);
        K.mu[k] = T(I.mu_[k]);
        K.lam[k] = T(I.lam[k]);
        K.cp[k] = T(I.cp[k]);
        K.chi[k] = T(I.chi[k]);
    }
    for (int w = 0; w < 4; w++) {
        K.tval[w] = T(I.tval[w]);
        K.wet[w] = T(I.wet[w]);
    }
    K.latent = T(I.latent);
    K.tm = T(I.tm);
    K.tl = T(I.tl);
    K.dx = T(I.dx);
    K.dt = T(I.dt);
    K.cpref = T(I.cpref);
    K.qg = T(I.qg);
    K.tau_g = T(I.tau_g);
    K.beta = T(I.beta);
    K.kappa = T(I.kappa);
    K.mu0 = T(I.mu0);
    K.h0x = T(I.h0x);
    K.h0y = T(I.h0y);
    K.vc = T(I.vc);
    K.grav[0] = T(I.grav[0]);
    K.grav[1] = T(I.grav[1]);
    K.idx = T(1.0 / I.dx);
    K.inv2dx = T(1.0 / (2.0 * I.dx));
    K.idx2 = T(1.0 / (I.dx * I.dx));
    K.i_halfdx = T(2.0 / I.dx);
    K.idt = T(1.0 / I.dt);
    K.mag_kdt = T(I.mag_kdt);
    K.tauf_k = T(3.0 / I.dts);
    K.tauh_k = T(3.0 / (I.cpref * I.dts));
}

// observables of one instance from its FP64 reduction results
int fill_observables(const lbfs_params& p, double t, int64_t step, double vol0, const double* r,
                     lbfs_observables* o)
{
    const double dA = p.dx * p.dx;
    std::memset(o, 0, sizeof *o);
    o->t = t;
    o->step = step;
    o->volume = r[RES_CT] * dA;
    o->volume0 = vol0;
    o->liquid_fraction = r[RES_CT] > 0.0 ? r[RES_CTFL] / r[RES_CT] : 0.0;
    o->solid_ratio = vol0 > 0.0 ? r[RES_FS] * dA / vol0 : 0.0;
    o->mag_residual = std::sqrt(r[RES_MAGR2]);
    o->umax = r[RES_UMAX];
    o->umax_drop = r[RES_UDROP];
    o->height = r[RES_HEIGHT] * p.dx;
    o->solid_height = r[RES_SOLIDH] * p.dx;
    o->wall_heat = r[RES_HEAT];
    // Eq. 50 with the liquid properties and the initial radius R0
    const double alpha_l = p.lambda[1] / (p.rho[1] * p.cp[1]);
    o->fourier = alpha_l * t / (p.drop_radius * p.drop_radius);
    o->peclet = o->umax_drop * 2.0 * p.drop_radius / alpha_l;
    if (r[RES_CT] > 0.0) {
        const double S = r[RES_CT], cx = r[RES_MX] / S, cy = r[RES_MY] / S;
        const double vxx = std::max(r[RES_MXX] / S - cx * cx, 0.0), vyy = std::max(r[RES_MYY] / S - cy * cy, 0.0);
        const double vxy = r[RES_MXY] / S - cx * cy;
        const double mean = 0.5 * (vxx + vyy), dev = std::sqrt(0.25 * (vxx - vyy) * (vxx - vyy) + vxy * vxy);
        o->centroid_x = cx;
        o->centroid_y = cy;
        o->semi_axis_x = 2.0 * std::sqrt(vxx);
        o->semi_axis_y = 2.0 * std::sqrt(vyy);
        o->semi_axis_major = 2.0 * std::sqrt(mean + dev);
        o->semi_axis_minor = 2.0 * std::sqrt(std::max(mean - dev, 0.0));
        double ang = 0.5 * std::atan2(2.0 * vxy, vxx - vyy) * 180.0 / M_PI;
        if (ang <= -90.0) ang += 180.0;
        o->major_axis_deg = ang;
    }
    o->nonfinite = r[RES_NONFINITE] != 0.0 || !std::isfinite(r[RES_CT]) ? 1 : 0;
    return o->nonfinite ? LBFS_E_NONFINITE : LBFS_OK;
}

}  // namespace

struct lbfs_solver {
    lbfs_params p;
    Layout L;
    hipStream_t stream = nullptr;
    char* base = nullptr;
    DevInst hinst{};
    DevInst* dinst = nullptr;
    Tile* dtiles_pt = nullptr;
    Exec E;                              // launches over this instance's own tiles
    bool batched = false;                // owned by a batch: stepped only by the batch
    int phi_field() const { return E.phase ? 17 : 15; }
    double* hres = nullptr;      // pinned copy of the results
    void* staging = nullptr;     // pinned field staging (nx*ny elements of 8 bytes)
    double t = 0.0;
    int64_t step = 0;
    double vol0 = 0.0;
    bool stepped_since_observe = false;  // the observables must be reduced again
    bool* owner_stale = nullptr;         // a batch member: its batch's flag of the same kind
    bool* owner_mu = nullptr;            // a batch member: its batch's permeability flag
    MgCtx mg;                            // multigrid plan (built on first use)
    void* field(int k) const { return base + L.off_fields + L.field_bytes * (size_t)k; }
    bool f64() const { return p.precision == LBFS_FP64; }
    // field k of the state (0-14: W, W1, W2; 15-17: phi[0], S, phi[1]), with the order
    // parameter of W, W1 and W2 where it is stored, and its element size
    static bool is_c(int k) { return k < 15 && k % 5 == 4; }
    void* sfield(int k) const
    {
        return is_c(k) && !f64() ? base + L.off_cfields + L.cfield_bytes * (size_t)(k / 5) : field(k);
    }
    size_t sesize(int k) const { return is_c(k) ? sizeof(double) : L.esize; }
};

// a failed HIP call: with LBFS_DEBUG=1 in the environment, name it on stderr
static bool hip_failed(hipError_t e, const char* expr, int line)
{
    if (e == hipSuccess) return false;
    static const int debug = [] {
        const char* v = std::getenv("LBFS_DEBUG");
        return v && v[0] == '1' ? 1 : 0;
    }();
    if (debug) std::fprintf(stderr, "lbfs: %s failed (lbfs_api.hip:%d): %s\n", expr, line, hipGetErrorString(e));
    return true;
}
#define HIPFAIL(x) hip_failed((x), #x, __LINE__)
#define HIPCHK(x)                                  \
    do {                                           \
        if (HIPFAIL(x)) return LBFS_E_DEVICE;      \
    } while (0)

namespace {

// Multigrid plan of a solver: levels halve each side (rounding up) down to at most
// MG_COARSE cells a side; the arrays of every level live in the ten stage fields.
int mg_plan(lbfs_solver* s)
{
    if (s->mg.L > 0) return LBFS_OK;
    if (s->p.periodic[0] || s->p.periodic[1]) return LBFS_E_INVAL;
    MgCtx& M = s->mg;
    const size_t es = s->L.esize;
    size_t off = 0;
    auto take = [&](size_t n) {
        const size_t o = off;
        off += (n + 63) / 64 * 64;   // 256-byte aligned in FP32
        return o;
    };
    int nx = s->p.nx, ny = s->p.ny;
    int L = 0;
    int w = 1, lx = 1, ly = 1;
    while (true) {
        if (L >= 24) return LBFS_E_INVAL;
        M.nx[L] = nx;
        M.ny[L] = ny;
        M.w[L] = w;
        M.lastx[L] = lx;
        M.lasty[L] = ly;
        M.wx[L] = take((size_t)(nx + 1) * ny);
        M.wy[L] = take((size_t)nx * (ny + 1));
        M.f[L] = take((size_t)nx * ny);
        M.u[L] = L == 0 ? 0 : take((size_t)nx * ny);
        L++;
        if (std::max(nx, ny) <= MG_COARSE) break;
        // the last coarse cell covers the last two fine cells, or only the last one
        lx = nx % 2 == 0 ? w + lx : lx;
        ly = ny % 2 == 0 ? w + ly : ly;
        w *= 2;
        nx = (nx + 1) / 2;
        ny = (ny + 1) / 2;
    }
    if (off * es > 10 * s->L.field_bytes) return LBFS_E_NOMEM;   // (never for grids of 4 x 4 and up)
    M.L = L;
    M.scratch = static_cast<char*>(s->field(5));
    M.phi[0] = s->field(15);
    M.phi[1] = s->field(17);
    M.pitch = s->L.pitch;
    M.fixed_walls = 0;
    for (int w = 0; w < 4; w++)
        if (s->p.mag_bc[w]) M.fixed_walls |= 1 << w;
    s->E.mg = &s->mg;
    return LBFS_OK;
}

// residual of the magnetic system of the current state, synchronously
int mag_residual_now(lbfs_solver* s, double* out)
{
    HIPCHK(exec_mag(s->E, 0, 1.0, 1));
    HIPCHK(launch_reduce(s->dinst, 1, s->stream));
    HIPCHK(hipMemcpyAsync(s->hres, s->hinst.result, sizeof(double) * NRES, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    *out = std::sqrt(s->hres[RES_MAGR2]);
    return LBFS_OK;
}

double phi_applied(const lbfs_params& p, int i, int j)
{
    const double th = p.field_angle_deg * M_PI / 180.0;
    const double x = (i + 0.5) * p.dx, y = (j + 0.5) * p.dx;
    return -p.h0 * (x * std::cos(th) + y * std::sin(th));
}

int field_index(int field)
{
    switch (field) {
    case LBFS_FIELD_HE: return 0;
    case LBFS_FIELD_P: return 1;
    case LBFS_FIELD_MX: return 2;
    case LBFS_FIELD_MY: return 3;
    case LBFS_FIELD_C: return 4;
    case LBFS_FIELD_PHI: return -2;   // current potential buffer
    case LBFS_FIELD_S: return 16;
    default: return -1;
    }
}

int copy_field_out(lbfs_solver* s, int k, double* host)
{
    const size_t es = s->sesize(k), nx = s->p.nx, ny = s->p.ny;
    HIPCHK(hipMemcpy2DAsync(s->staging, nx * es, s->sfield(k), (size_t)s->L.pitch * es, nx * es, ny,
                            hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    for (size_t q = 0; q < nx * ny; q++)
        host[q] = es == 8 ? static_cast<double*>(s->staging)[q] : (double)static_cast<float*>(s->staging)[q];
    return LBFS_OK;
}

// the state was written from outside a step: the next observe reduces it again (for a
// batch member, the batch's next observe too)
void mark_written(lbfs_solver* s)
{
    s->stepped_since_observe = true;
    if (s->owner_stale) *s->owner_stale = true;
    // (and the next magnetic phase computes the permeability itself)
    s->E.mu_ready = false;
    if (s->owner_mu) *s->owner_mu = false;
}

int copy_field_in(lbfs_solver* s, int k, const double* host)
{
    const size_t es = s->sesize(k), nx = s->p.nx, ny = s->p.ny;
    for (size_t q = 0; q < nx * ny; q++) {
        if (es == 8) static_cast<double*>(s->staging)[q] = host[q];
        else static_cast<float*>(s->staging)[q] = (float)host[q];
    }
    HIPCHK(hipMemcpy2DAsync(s->sfield(k), (size_t)s->L.pitch * es, s->staging, nx * es, nx * es, ny,
                            hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    mark_written(s);
    return LBFS_OK;
}

}  // namespace

extern "C" {

int lbfs_params_default(lbfs_params* p, int32_t nx, int32_t ny, int32_t precision)
{
    if (!p) return LBFS_E_INVAL;
    std::memset(p, 0, sizeof *p);
    p->abi_version = LBFS_ABI_VERSION;
    p->nx = nx;
    p->ny = ny;
    p->precision = precision;
    p->dx = 1.0;
    p->dt = 0.5;
    p->dt_stream = 0.5;
    const double rho_g = 0.1;
    const double rho[3] = {1450.0 / 1580.0, 1.0, rho_g};
    const double mu[3] = {0.02, 0.02, 0.002};
    const double cp[3] = {1670.0 / 3000.0, 1.0, 1.0};
    const double lam[3] = {0.05 * 2.32 / 0.72, 0.05, 0.4 * rho_g};
    const double chi[3] = {1.0, 1.0, 0.0};
    for (int k = 0; k < 3; k++) {
        p->rho[k] = rho[k]; p->mu[k] = mu[k]; p->cp[k] = cp[k]; p->lambda[k] = lam[k]; p->chi[k] = chi[k];
    }
    p->latent = 10.0;
    p->t_melt = 0.0;
    p->t_liquidus = 0.0;
    p->t_init = 0.0;
    p->mu0 = 1.0;
    p->h0 = 0.0;
    p->field_angle_deg = 90.0;
    p->sigma = 0.005;
    p->xi = 4.0;
    p->mobility = 0.05;
    p->tau_g = 1.0;
    p->drop_cx = 0.5 * nx;
    p->drop_cy = 0.0;
    p->drop_radius = 0.25 * nx;
    p->init_kind = LBFS_INIT_DROPLET;
    p->c_init = 1.0;
    p->thermal_bc[2] = LBFS_TBC_FIXED;
    p->thermal_val[2] = -1.0;
    for (int w = 0; w < 4; w++) {
        p->mag_bc[w] = LBFS_MBC_FIXED;
        p->contact_angle_deg[w] = 90.0;
    }
    p->sweeps = 4;
    p->sor_omega = 1.0;
    p->mag_method = LBFS_MAG_SWEEPS;
    p->mag_lbfs_d = 1.0;
    p->mag_lbfs_dtau = 0.0;
    p->mag_max_iters = 0;
    p->mag_tol = 0.0;
    p->init_omega = 0.0;
    p->init_tol = precision == LBFS_FP64 ? 1e-9 : 1e-4;
    p->init_max = 20 * (nx > ny ? nx : ny) + 1000;
    p->init_check = 50;
    return LBFS_OK;
}

int lbfs_params_from_dimless(lbfs_params* p, double ste, double t_wall, double bo_m, double angle_deg)
{
    if (!p || !finite_pos(ste) || !std::isfinite(t_wall) || !std::isfinite(bo_m) || bo_m < 0.0 ||
        !finite_pos(p->drop_radius) || !finite_pos(p->mu0) || !std::isfinite(angle_deg))
        return LBFS_E_INVAL;
    p->latent = p->cp[1] * (p->t_melt - t_wall) / ste;       // Ste = Cp_l (Tm - Tw) / L
    p->h0 = std::sqrt(bo_m * p->sigma / (p->mu0 * 2.0 * p->drop_radius));   // Bo_m = mu0 H^2 D / sigma
    p->field_angle_deg = angle_deg;
    p->thermal_bc[2] = LBFS_TBC_FIXED;
    p->thermal_val[2] = t_wall;
    return LBFS_OK;
}

size_t lbfs_state_bytes(const lbfs_params* p)
{
    if (validate(p) != LBFS_OK) return 0;
    return make_layout(p).total;
}

static void destroy_solver(lbfs_solver* s);

// tile lists of the given shapes into the solver's own segments; drops the graphs
// the sweeps can run inside stage 1: a fixed count within one launch's halo
static bool fusable(const lbfs_params& p)
{
    return p.mag_method == LBFS_MAG_SWEEPS && p.mag_max_iters == 0 && p.sweeps <= MAG_KMAX;
}

// stage and magnetic tile shapes; mi == NMAG_SHAPES runs the sweeps inside stage 1 and
// keeps the magnetic tiles (still used by the initial solve and lbfs_mag_sweeps)
static int apply_shapes(lbfs_solver* s, int si, int mi)
{
    if (si < 0 || si >= NSTAGE_SHAPES || mi < 0 || mi > NMAG_SHAPES) return LBFS_E_INVAL;
    if (mi == NMAG_SHAPES && !fusable(s->p)) return LBFS_E_INVAL;
    const bool fuse = mi == NMAG_SHAPES;
    if (fuse) mi = s->E.mag_shape;
    std::vector<Tile> ts, tm;
    append_tiles(ts, 0, s->p.nx, s->p.ny, stage_shape(s->f64(), si));
    append_tiles(tm, 0, s->p.nx, s->p.ny, MAG_SHAPES[mi], true);
    HIPCHK(hipStreamSynchronize(s->stream));   // launches in flight read the old lists
    exec_drop_graphs(s->E);
    Exec& E = s->E;
    s->hinst.ntile_stage = (int)ts.size();
    s->hinst.ntile_mag = (int)tm.size();
    HIPCHK(hipMemcpyAsync(const_cast<Tile*>(E.tiles_stage), ts.data(), sizeof(Tile) * ts.size(),
                          hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(const_cast<Tile*>(E.tiles_mag), tm.data(), sizeof(Tile) * tm.size(), hipMemcpyHostToDevice,
                          s->stream));
    HIPCHK(hipMemcpyAsync(s->dinst, &s->hinst, sizeof(DevInst), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    E.stage_shape = si;
    E.mag_shape = mi;
    E.fused = fuse;
    E.nstage = (int)ts.size();
    E.nmag = (int)tm.size();
    s->stepped_since_observe = true;
    return LBFS_OK;
}

// the parameters of an instance in its descriptor (dt and dt_stream already resolved),
// with the coefficient blocks of both precisions
static void fill_params(DevInst& I, const lbfs_params& p, int pitch)
{
    I.nx = p.nx;
    I.ny = p.ny;
    I.pitch = pitch;
    I.per_x = p.periodic[0];
    I.per_y = p.periodic[1];
    for (int w = 0; w < 4; w++) {
        I.tbc[w] = p.thermal_bc[w];
        I.mbc[w] = p.mag_bc[w];
        I.tval[w] = p.thermal_val[w];
        // wetting: n.grad C = -(4/xi) cos(theta) C (1 - C) at the wall (exactly the
        // mirror at 90 degrees)
        I.wet[w] = p.contact_angle_deg[w] == 90.0 ? 0.0 : 4.0 / p.xi * std::cos(p.contact_angle_deg[w] * M_PI / 180.0);
    }
    int col = (int)std::floor(p.drop_cx / p.dx);
    I.col_height = col < 0 ? 0 : (col > p.nx - 1 ? p.nx - 1 : col);
    I.heat_on = (!p.periodic[1] && p.thermal_bc[2] == LBFS_TBC_FIXED) ? 1 : 0;
    for (int k = 0; k < 3; k++) {
        I.rho[k] = p.rho[k]; I.mu_[k] = p.mu[k]; I.lam[k] = p.lambda[k]; I.cp[k] = p.cp[k]; I.chi[k] = p.chi[k];
    }
    I.latent = p.latent;
    I.tm = p.t_melt;
    I.tl = p.t_liquidus;
    I.dx = p.dx;
    I.dt = p.dt;
    I.dts = p.dt_stream;
    I.cpref = 0.5 * (p.cp[0] + p.cp[1]);
    I.qg = p.mobility / ((p.tau_g - 0.5) * p.dt_stream);   // M_c = (tau_g - 1/2) Q_g delta_t
    I.tau_g = p.tau_g;
    I.beta = 12.0 * p.sigma / p.xi;
    I.kappa = 1.5 * p.xi * p.sigma;
    I.mu0 = p.mu0;
    const double th = p.field_angle_deg * M_PI / 180.0;
    I.h0x = p.h0 * std::cos(th);
    I.h0y = p.h0 * std::sin(th);
    I.xi = p.xi;
    I.grav[0] = p.gravity[0];
    I.grav[1] = p.gravity[1];
    I.vc = 1.0 - p.rho[0] / p.rho[1];
    {
        // the automatic pseudo-time step dx^2 / (4 D mu_max): every row of the discrete
        // operator sums in absolute value to at most 8 D mu_max / dx^2, and SSP-RK3 is
        // stable on the negative real axis to about -2.51; the mixture permeability
        // never exceeds that of the most permeable phase
        double mmax = 1.0 + p.chi[0];
        for (int k = 1; k < 3; k++) mmax = std::max(mmax, 1.0 + p.chi[k]);
        I.mag_kdt = p.mag_lbfs_dtau > 0.0 ? p.mag_lbfs_d * p.mag_lbfs_dtau / (p.dx * p.dx)
                                           : 1.0 / (4.0 * p.mu0 * mmax);
    }
    I.mag_tol = p.mag_tol;
    fill_coef(I.cf, I);
    fill_coef(I.cd, I);
}

static int init_solver(const lbfs_params* p, void* dev_buf, size_t bytes, void* stream, lbfs_solver** out)
{
    if (!out) return LBFS_E_INVAL;
    *out = nullptr;
    const int v = validate(p);
    if (v != LBFS_OK) return v;
    if (!dev_buf) return LBFS_E_INVAL;
    const Layout L = make_layout(p);
    if (bytes < L.total) return LBFS_E_NOMEM;

    lbfs_solver* s = new (std::nothrow) lbfs_solver();
    if (!s) return LBFS_E_NOMEM;
    s->p = *p;
    if (s->p.dt == 0.0) s->p.dt = auto_dt(*p);
    if (s->p.dt_stream == 0.0) s->p.dt_stream = 0.5 * p->dx;
    if (s->p.init_check == 0) s->p.init_check = 50;
    s->L = L;
    s->stream = static_cast<hipStream_t>(stream);
    s->base = reinterpret_cast<char*>(align_up(reinterpret_cast<uintptr_t>(dev_buf), ALIGN));
    s->dinst = reinterpret_cast<DevInst*>(s->base + L.off_inst);
    s->dtiles_pt = reinterpret_cast<Tile*>(s->base + L.off_tpt);
    Exec& E = s->E;
    E.f64 = p->precision == LBFS_FP64;
    E.sweeps = p->sweeps;
    E.omega = p->sor_omega;
    E.mag_method = p->mag_method;
    E.mag_chunks = p->mag_max_iters > 0 ? (p->mag_max_iters + p->sweeps - 1) / p->sweeps : 1;
    E.stream = s->stream;
    E.dinst = s->dinst;
    E.ninst = 1;
    E.tiles_stage = reinterpret_cast<Tile*>(s->base + L.off_tstage);
    E.tiles_mag = reinterpret_cast<Tile*>(s->base + L.off_tmag);
    auto fail = [&](int code) {
        destroy_solver(s);
        return code;
    };
    if (hipHostMalloc(&s->hres, sizeof(double) * NRES, hipHostMallocDefault) != hipSuccess) return fail(LBFS_E_DEVICE);
    if (hipHostMalloc(&s->staging, (size_t)p->nx * p->ny * 8, hipHostMallocDefault) != hipSuccess)
        return fail(LBFS_E_DEVICE);

    // descriptor
    DevInst& I = s->hinst;
    std::memset(&I, 0, sizeof I);
    for (int k = 0; k < 5; k++) {
        I.W[k] = s->sfield(k);
        I.W1[k] = s->sfield(5 + k);
        I.W2[k] = s->sfield(10 + k);
    }
    I.phi[0] = s->field(15);
    I.phi[1] = s->field(17);
    I.S = s->field(16);
    for (int k = 0; k < 3; k++)
        I.kf[k] = s->f64() ? static_cast<void*>(s->base + L.off_cfields + L.field_bytes * (size_t)k)
                           : s->field(4 + 5 * k);
    I.part = reinterpret_cast<double*>(s->base + L.off_part);
    I.mpart = reinterpret_cast<double*>(s->base + L.off_mpart);
    I.result = reinterpret_cast<double*>(s->base + L.off_res);
    fill_params(I, s->p, L.pitch);

    std::vector<Tile> tp;
    append_tiles(tp, 0, p->nx, p->ny, TileShape{PT_TX, PT_TY, PT_TX * PT_TY});
    if (hipMemcpyAsync(s->dtiles_pt, tp.data(), sizeof(Tile) * tp.size(), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemsetAsync(s->base + L.off_part, 0, L.off_fields - L.off_part, s->stream) != hipSuccess ||
        hipMemsetAsync(s->base + L.off_fields, 0, L.total - ALIGN - L.off_fields, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return fail(LBFS_E_DEVICE);
    // default shapes by precision and grid size
    if (apply_shapes(s, default_stage_shape(s->f64(), (size_t)p->nx * p->ny),
                     default_mag_shape((size_t)p->nx * p->ny)) != LBFS_OK)
        return fail(LBFS_E_DEVICE);

    hipError_t e = s->f64()
        ? launch_init_fields<double>(s->dinst, s->dtiles_pt, L.ntile_pt(), p->init_kind, p->c_init, p->t_init,
                                     p->drop_cx, p->drop_cy, p->drop_radius, s->stream)
        : launch_init_fields<float>(s->dinst, s->dtiles_pt, L.ntile_pt(), p->init_kind, p->c_init, p->t_init,
                                    p->drop_cx, p->drop_cy, p->drop_radius, s->stream);
    if (e != hipSuccess) return fail(LBFS_E_DEVICE);

    if (p->mag_method == LBFS_MAG_MULTIGRID && mg_plan(s) != LBFS_OK) return fail(LBFS_E_INVAL);
    // converge the magnetic potential (Table 1, before the main loop)
    double r0 = 0.0;
    if (mag_residual_now(s, &r0) != LBFS_OK) return fail(LBFS_E_DEVICE);
    double om = p->init_omega;
    if (om <= 0.0) {
        const int nmax = p->nx > p->ny ? p->nx : p->ny;
        om = 2.0 / (1.0 + std::sin(M_PI / nmax));
    }
    int used = 0;
    double r = r0;
    while (r0 > 0.0 && used < p->init_max && r > p->init_tol * r0) {
        int k = s->p.init_check;
        if (used + k > p->init_max) k = p->init_max - used;
        if (p->mag_method == LBFS_MAG_MULTIGRID) {
            // one cycle per check (init_max still counts sweeps: a cycle counts as init_check)
            if (exec_mg(E, 1, 0) != hipSuccess) return fail(LBFS_E_DEVICE);
        } else if (exec_mag(E, k, om, 0) != hipSuccess) {
            return fail(LBFS_E_DEVICE);
        }
        used += k;
        const double r_prev = r;
        if (mag_residual_now(s, &r) != LBFS_OK) return fail(LBFS_E_DEVICE);
        if (!std::isfinite(r)) return fail(LBFS_E_NONFINITE);
        if (r > 0.98 * r_prev) break;   // stagnated at the round-off floor of the precision
    }
    // observables of the initial state (also the reference volume A0)
    if (exec_state_partials(E) != hipSuccess || launch_reduce(s->dinst, 1, s->stream) != hipSuccess ||
        hipMemcpyAsync(s->hres, I.result, sizeof(double) * NRES, hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return fail(LBFS_E_DEVICE);
    s->vol0 = s->hres[RES_CT] * p->dx * p->dx;
    s->hres[RES_MAGR2] = r * r;
    const char* ng = std::getenv("LBFS_NO_GRAPH");
    // graph replays pay where the kernels are short enough for the host's launches to
    // lag (256^2: 25.7 against 26.7 us per step); from about 2^19 cells on direct launches
    // are as fast or faster (1024^2: 133.3 against 135.1 us), so large grids launch
    // directly unless LBFS_GRAPH=1
    const char* gf = std::getenv("LBFS_GRAPH");
    const bool small = (int64_t)p->nx * p->ny < ((int64_t)1 << 19);
    E.use_graph = s->stream != nullptr && !(ng && ng[0] == '1') && (small || (gf && gf[0] == '1'));
    exec_set_graph_steps(E, graph_steps_setting());
    *out = s;
    return LBFS_OK;
}

int lbfs_init(const lbfs_params* p, void* dev_buf, size_t bytes, void* stream, lbfs_solver** out)
{
    return init_solver(p, dev_buf, bytes, stream, out);
}

int lbfs_step(lbfs_solver* s, int32_t nsteps)
{
    if (!s || s->batched) return LBFS_E_STATE;
    if (nsteps < 0) return LBFS_E_INVAL;
    for (int n = 0; n < nsteps;) {
        const int k = exec_run_steps(s->E, nsteps - n);
        if (k == 0) return LBFS_E_DEVICE;
        for (int q = 0; q < k; q++) s->t += s->p.dt;
        s->step += k;
        s->stepped_since_observe = true;
        n += k;
    }
    return LBFS_OK;
}

int lbfs_prepare(lbfs_solver* s)
{
    if (!s || s->batched) return LBFS_E_STATE;
    HIPCHK(exec_prepare(s->E));
    return LBFS_OK;
}

int lbfs_step_profiled_start(lbfs_solver* s, int32_t nsteps, int32_t sample_every)
{
    if (!s || s->batched) return LBFS_E_STATE;
    if (nsteps < 0 || sample_every < 1) return LBFS_E_INVAL;
    return exec_profiled_start(s->E, nsteps, sample_every, [&] {
        s->t += s->p.dt;
        s->step += 1;
        s->stepped_since_observe = true;
    });
}

int lbfs_profile_result(lbfs_solver* s, double* kernel_ms, int32_t* launches)
{
    if (!s || s->batched) return LBFS_E_STATE;
    if (!kernel_ms || !launches) return LBFS_E_INVAL;
    return exec_profiled_result(s->E, kernel_ms, launches);
}

int lbfs_step_profiled(lbfs_solver* s, int32_t nsteps, int32_t sample_every, double* kernel_ms,
                       int32_t* launches)
{
    if (!s || s->batched) return LBFS_E_STATE;
    if (nsteps < 0 || sample_every < 1 || !kernel_ms || !launches) return LBFS_E_INVAL;
    const int rc = lbfs_step_profiled_start(s, nsteps, sample_every);
    return rc == LBFS_OK ? lbfs_profile_result(s, kernel_ms, launches) : rc;
}

int lbfs_observe(lbfs_solver* s, lbfs_observables* o)
{
    if (!s || !o) return s ? LBFS_E_INVAL : LBFS_E_STATE;
    if (s->stepped_since_observe) {
        HIPCHK(exec_state_partials(s->E));
        HIPCHK(launch_reduce(s->dinst, 1, s->stream, s->E.mres_stage));
        HIPCHK(hipMemcpyAsync(s->hres, s->hinst.result, sizeof(double) * NRES, hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        s->stepped_since_observe = false;
    }
    return fill_observables(s->p, s->t, s->step, s->vol0, s->hres, o);
}

int lbfs_rhs(lbfs_solver* s, double* host_R)
{
    if (!s) return LBFS_E_STATE;
    if (!host_R) return LBFS_E_INVAL;
    HIPCHK(exec_stage(s->E, 0));
    const size_t n = (size_t)s->p.nx * s->p.ny;
    for (int k = 0; k < 5; k++) {
        const int rc = copy_field_out(s, 5 + k, host_R + k * n);
        if (rc != LBFS_OK) return rc;
    }
    return LBFS_OK;
}

int lbfs_mag_sweeps(lbfs_solver* s, int32_t nsweeps, double omega, double* residual)
{
    if (!s) return LBFS_E_STATE;
    if (s->batched) return LBFS_E_STATE;   // would flip the potential parity of one batch member
    if (nsweeps < 0 || !(omega > 0.0 && omega < 2.0)) return LBFS_E_INVAL;
    HIPCHK(exec_mag(s->E, nsweeps, omega, 0));
    double r = 0.0;
    const int rc = mag_residual_now(s, &r);
    if (rc != LBFS_OK) return rc;
    if (residual) *residual = r;
    return LBFS_OK;
}

int lbfs_mag_pseudo_steps(lbfs_solver* s, int32_t nsteps, double* residual)
{
    if (!s) return LBFS_E_STATE;
    if (s->batched) return LBFS_E_STATE;
    if (nsteps < 0) return LBFS_E_INVAL;
    HIPCHK(exec_mag_lbfs(s->E, nsteps, 0));
    double r = 0.0;
    const int rc = mag_residual_now(s, &r);
    if (rc != LBFS_OK) return rc;
    if (residual) *residual = r;
    return LBFS_OK;
}

int lbfs_mag_multigrid(lbfs_solver* s, int32_t ncycles, double* residual)
{
    if (!s) return LBFS_E_STATE;
    if (s->batched) return LBFS_E_STATE;
    if (ncycles < 0 || ncycles > 10000) return LBFS_E_INVAL;
    const int rc = mg_plan(s);
    if (rc != LBFS_OK) return rc;
    exec_drop_graphs(s->E);   // (a plan built now changes no captured step; kept simple)
    HIPCHK(exec_mg(s->E, ncycles, 0));
    double r = 0.0;
    const int rr = mag_residual_now(s, &r);
    if (rr != LBFS_OK) return rr;
    if (residual) *residual = r;
    return LBFS_OK;
}

int lbfs_wall_heat_profile(lbfs_solver* s, double* host_q, size_t n)
{
    if (!s) return LBFS_E_STATE;
    if (!host_q || n != (size_t)s->p.nx) return LBFS_E_INVAL;
    // the stage-1 field is free between steps: FP64 scratch for the nx values
    double* out = static_cast<double*>(s->field(5));
    HIPCHK(s->f64() ? launch_wall_profile<double>(s->dinst, s->p.nx, out, s->stream)
                    : launch_wall_profile<float>(s->dinst, s->p.nx, out, s->stream));
    HIPCHK(hipMemcpyAsync(s->staging, out, n * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    std::memcpy(host_q, s->staging, n * sizeof(double));
    return LBFS_OK;
}

int lbfs_read_field(lbfs_solver* s, int32_t field, double* host, size_t n)
{
    if (!s) return LBFS_E_STATE;
    const size_t nn = (size_t)s->p.nx * s->p.ny;
    if (!host || n != nn) return LBFS_E_INVAL;
    if (field == LBFS_FIELD_T || field == LBFS_FIELD_FL) {
        const int np = s->L.ntile_pt();
        HIPCHK(s->f64() ? launch_derived<double>(s->dinst, s->dtiles_pt, np, s->stream)
                        : launch_derived<float>(s->dinst, s->dtiles_pt, np, s->stream));
        return copy_field_out(s, field == LBFS_FIELD_T ? 5 : 6, host);
    }
    int k = field_index(field);
    if (k == -2) k = s->phi_field();
    if (k < 0) return LBFS_E_INVAL;
    const int rc = copy_field_out(s, k, host);
    if (rc != LBFS_OK) return rc;
    if (field == LBFS_FIELD_PHI)
        for (int j = 0; j < s->p.ny; j++)
            for (int i = 0; i < s->p.nx; i++) host[(size_t)j * s->p.nx + i] += phi_applied(s->p, i, j);
    return LBFS_OK;
}

int lbfs_write_field(lbfs_solver* s, int32_t field, const double* host, size_t n)
{
    if (!s) return LBFS_E_STATE;
    const size_t nn = (size_t)s->p.nx * s->p.ny;
    if (!host || n != nn) return LBFS_E_INVAL;
    int k = field_index(field);
    if (k == -2) k = s->phi_field();
    if (k < 0) return LBFS_E_INVAL;
    if (field == LBFS_FIELD_PHI) {
        std::vector<double> d(host, host + nn);
        for (int j = 0; j < s->p.ny; j++)
            for (int i = 0; i < s->p.nx; i++) d[(size_t)j * s->p.nx + i] -= phi_applied(s->p, i, j);
        return copy_field_in(s, k, d.data());
    }
    return copy_field_in(s, k, host);
}

int lbfs_set_time(lbfs_solver* s, double t, int64_t step)
{
    if (!s) return LBFS_E_STATE;
    if (!std::isfinite(t) || step < 0) return LBFS_E_INVAL;
    s->t = t;
    s->step = step;
    return LBFS_OK;
}

namespace {
struct CkptHeader {
    uint32_t magic, abi;
    int32_t nx, ny, precision, pad;
    double t, vol0;
    int64_t step;
};
constexpr int CKPT_FIELDS[7] = {0, 1, 2, 3, 4, -2, 16};   // -2: current potential buffer
// element size of checkpoint field q (the order parameter is FP64 in both precisions)
size_t ckpt_esize(const lbfs_solver* s, int q) { return CKPT_FIELDS[q] == 4 ? sizeof(double) : s->L.esize; }
}  // namespace

size_t lbfs_checkpoint_bytes(const lbfs_solver* s)
{
    if (!s) return 0;
    size_t b = sizeof(CkptHeader);
    for (int q = 0; q < 7; q++) b += (size_t)s->p.nx * s->p.ny * ckpt_esize(s, q);
    return b;
}

int lbfs_save_state(lbfs_solver* s, void* host, size_t bytes)
{
    if (!s) return LBFS_E_STATE;
    if (!host || bytes < lbfs_checkpoint_bytes(s)) return LBFS_E_INVAL;
    CkptHeader h{CKPT_MAGIC, LBFS_ABI_VERSION, s->p.nx, s->p.ny, s->p.precision, 0, s->t, s->vol0, s->step};
    std::memcpy(host, &h, sizeof h);
    char* dst = static_cast<char*>(host) + sizeof h;
    for (int q = 0; q < 7; q++) {
        const size_t es = ckpt_esize(s, q), row = (size_t)s->p.nx * es, fb = row * s->p.ny;
        const int f = CKPT_FIELDS[q] == -2 ? s->phi_field() : CKPT_FIELDS[q];
        HIPCHK(hipMemcpy2DAsync(s->staging, row, s->sfield(f), (size_t)s->L.pitch * es, row, s->p.ny,
                                hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        std::memcpy(dst, s->staging, fb);
        dst += fb;
    }
    return LBFS_OK;
}

int lbfs_load_state(lbfs_solver* s, const void* host, size_t bytes)
{
    if (!s) return LBFS_E_STATE;
    if (!host || bytes < lbfs_checkpoint_bytes(s)) return LBFS_E_INVAL;
    CkptHeader h;
    std::memcpy(&h, host, sizeof h);
    if (h.magic != CKPT_MAGIC || h.abi != LBFS_ABI_VERSION || h.nx != s->p.nx || h.ny != s->p.ny ||
        h.precision != s->p.precision)
        return LBFS_E_INVAL;
    const char* src = static_cast<const char*>(host) + sizeof h;
    for (int q = 0; q < 7; q++) {
        const size_t es = ckpt_esize(s, q), row = (size_t)s->p.nx * es, fb = row * s->p.ny;
        std::memcpy(s->staging, src, fb);
        src += fb;
        const int f = CKPT_FIELDS[q] == -2 ? s->phi_field() : CKPT_FIELDS[q];
        HIPCHK(hipMemcpy2DAsync(s->sfield(f), (size_t)s->L.pitch * es, s->staging, row, row, s->p.ny,
                                hipMemcpyHostToDevice, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    s->t = h.t;
    s->step = h.step;
    s->vol0 = h.vol0;
    mark_written(s);
    return LBFS_OK;
}

static void destroy_solver(lbfs_solver* s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    exec_release(s->E);
    if (s->hres) (void)hipHostFree(s->hres);
    if (s->staging) (void)hipHostFree(s->staging);
    delete s;
}

}  // extern "C"

// ------------------------------------------------------------------ static scratch
//
// lbfs_step_fields works in this array: the stage fields W1 and W2, the second potential
// buffer, the descriptor, the tile lists and the residual partials of one instance. Each
// device that runs the library holds its own copy until the process ends. In host code
// the name is only a stand-in: the device address comes from hipGetSymbolAddress, once
// per device, and only that address is passed to kernels and copies.
static __device__ __align__(256) unsigned char scratch[LBFS_STATIC_SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mutex;
char* scratch_addr[SCRATCH_MAX_DEVICES] = {};

// device address of the current device's scratch (looked up on its first use)
int static_scratch(char** out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= SCRATCH_MAX_DEVICES) return LBFS_E_DEVICE;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_addr[dev]) {
        void* a = nullptr;
        if (hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)) != hipSuccess || !a) return LBFS_E_DEVICE;
        scratch_addr[dev] = static_cast<char*>(a);
    }
    *out = scratch_addr[dev];
    return LBFS_OK;
}

static_assert(sizeof(DevInst) <= 3072, "the descriptor travels as a kernel argument");
// the autotuners' timing arrays: every stage shape, then every magnetic shape and the
// fused variant, each within LBFS_MAX_SHAPES
static_assert(NSTAGE_SHAPES <= LBFS_MAX_SHAPES && NMAG_SHAPES < LBFS_MAX_SHAPES, "shape tables fit the ABI arrays");

// the descriptor into device memory without a host-to-device copy
__global__ void k_write_desc(DevInst d, DevInst* dst)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *dst = d;
}

// the tile list of one instance of ntiles = ntx x nty tiles (the list append_tiles gives)
__global__ void k_fill_tiles(Tile* out, int nx, int tw, int th, int ntiles, int blocked)
{
    const int i = blockIdx.x * blockDim.x + (int)threadIdx.x;
    if (i >= ntiles) return;
    const int ntx = (nx + tw - 1) / tw, nty = ntiles / ntx;
    int tx = i % ntx, ty = i / ntx;
    if (blocked) tile_at(i, ntx, nty, tw, th, tx, ty);
    out[i] = Tile{0, tx * tw, ty * th, ty * ntx + tx};
}

}  // namespace

extern "C" {

int lbfs_step_fields(const lbfs_params* p, void* const fields[7], int32_t nsteps, void* stream)
{
    if (!p || !fields) return LBFS_E_INVAL;
    const int v = validate(p);
    if (v != LBFS_OK) return v;
    if (nsteps < 0) return LBFS_E_INVAL;
    for (int k = 0; k < 7; k++)
        if (!fields[k]) return LBFS_E_INVAL;
    if (p->mag_method == LBFS_MAG_MULTIGRID || p->mag_max_iters > 0) return LBFS_E_INVAL;
    lbfs_params q = *p;
    if (q.dt == 0.0) q.dt = auto_dt(*p);
    if (q.dt_stream == 0.0) q.dt_stream = 0.5 * q.dx;
    const bool f64 = q.precision == LBFS_FP64;
    const size_t es = f64 ? 8 : 4, n = (size_t)q.nx * q.ny;
    // the tile shapes a solver of this size starts with
    const int sshape = default_stage_shape(f64, n), mshape = default_mag_shape(n);
    const TileShape SS = stage_shape(f64, sshape);
    const TileShape MS = MAG_SHAPES[mshape];
    const int nts = count_tiles(q.nx, q.ny, SS), ntm = count_tiles(q.nx, q.ny, MS);
    // layout of the scratch for this problem
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off = align_up(off + b, ALIGN);
        return o;
    };
    const size_t o_inst = take(sizeof(DevInst));
    const size_t o_ts = take(sizeof(Tile) * nts), o_tm = take(sizeof(Tile) * ntm);
    const size_t o_mpart = take(sizeof(double) * (std::max(nts, ntm) + 1));
    const size_t o_res = take(sizeof(double) * NRES);
    size_t o_w1[5], o_w2[5];
    for (int k = 0; k < 5; k++) o_w1[k] = take(n * (k == 4 ? sizeof(double) : es));
    for (int k = 0; k < 5; k++) o_w2[k] = take(n * (k == 4 ? sizeof(double) : es));
    const size_t o_phi1 = take(n * es);
    size_t o_kf[3];
    for (int k = 0; k < 3; k++) o_kf[k] = take(n * es);
    if (off > LBFS_STATIC_SCRATCH_BYTES) return LBFS_E_NOMEM;
    char* base = nullptr;
    const int rs = static_scratch(&base);
    if (rs != LBFS_OK) return rs;

    DevInst I;
    std::memset(&I, 0, sizeof I);
    for (int k = 0; k < 5; k++) {
        I.W[k] = fields[k];
        I.W1[k] = base + o_w1[k];
        I.W2[k] = base + o_w2[k];
    }
    I.phi[0] = fields[5];
    I.phi[1] = base + o_phi1;
    I.S = fields[6];
    for (int k = 0; k < 3; k++) I.kf[k] = base + o_kf[k];
    I.part = nullptr;   // (observables are not reduced here)
    I.mpart = reinterpret_cast<double*>(base + o_mpart);
    I.result = reinterpret_cast<double*>(base + o_res);
    I.ntile_stage = nts;
    I.ntile_mag = ntm;
    fill_params(I, q, q.nx);   // caller fields: row pitch nx

    hipStream_t st = static_cast<hipStream_t>(stream);
    DevInst* dinst = reinterpret_cast<DevInst*>(base + o_inst);
    Tile* ts = reinterpret_cast<Tile*>(base + o_ts);
    Tile* tm = reinterpret_cast<Tile*>(base + o_tm);
    hipLaunchKernelGGL(k_write_desc, dim3(1), dim3(64), 0, st, I, dinst);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_fill_tiles, dim3((nts + 255) / 256), dim3(256), 0, st, ts, q.nx, SS.tx, SS.ty, nts, 0);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_fill_tiles, dim3((ntm + 255) / 256), dim3(256), 0, st, tm, q.nx, MS.tx, MS.ty, ntm, 1);
    HIPCHK(hipGetLastError());

    Exec E;
    E.f64 = f64;
    E.stage_shape = sshape;
    E.mag_shape = mshape;
    E.sweeps = q.sweeps;
    E.omega = q.sor_omega;
    E.mag_method = q.mag_method;
    E.mag_chunks = 1;
    E.stream = st;
    E.dinst = dinst;
    E.ninst = 1;
    E.tiles_stage = ts;
    E.nstage = nts;
    E.tiles_mag = tm;
    E.nmag = ntm;
    E.phase = 0;
    E.use_graph = false;
    for (int k = 0; k < nsteps; k++) HIPCHK(exec_enqueue_step(E, k == nsteps - 1));
    // the potential ends in the caller's field
    if (E.phase != 0) HIPCHK(hipMemcpyAsync(fields[5], base + o_phi1, n * es, hipMemcpyDeviceToDevice, st));
    return LBFS_OK;
}

void lbfs_destroy(lbfs_solver* s)
{
    if (!s || s->batched) return;   // batch members are released by lbfs_batch_retire
    destroy_solver(s);
}

const char* lbfs_strerror(int status)
{
    switch (status) {
    case LBFS_OK: return "ok";
    case LBFS_E_INVAL: return "invalid argument or parameters";
    case LBFS_E_NOMEM: return "buffer too small or budget exhausted";
    case LBFS_E_NONFINITE: return "non-finite value in the state";
    case LBFS_E_DEVICE: return "HIP device call failed";
    case LBFS_E_STATE: return "call out of order";
    case LBFS_E_ABI: return "ABI version mismatch";
    default: return "unknown status";
    }
}

}  // extern "C"


// ------------------------------------------------------------------ tile shapes

namespace {

// mean duration (ms) of `reps` enqueues of f on the stream, after one untimed warm-up
template <typename F>
int time_launches(hipStream_t stream, int reps, F&& f, double* ms)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (HIPFAIL(hipEventCreate(&e0)) || HIPFAIL(hipEventCreate(&e1))) {
        if (e0) (void)hipEventDestroy(e0);
        return LBFS_E_DEVICE;
    }
    int rc = LBFS_OK;
    float t = 0.0f;
    if (HIPFAIL(f()) || HIPFAIL(hipEventRecord(e0, stream))) rc = LBFS_E_DEVICE;
    for (int k = 0; k < reps && rc == LBFS_OK; k++)
        if (HIPFAIL(f())) rc = LBFS_E_DEVICE;
    if (rc == LBFS_OK && (HIPFAIL(hipEventRecord(e1, stream)) || HIPFAIL(hipEventSynchronize(e1)) ||
                          HIPFAIL(hipEventElapsedTime(&t, e0, e1))))
        rc = LBFS_E_DEVICE;
    *ms = rc == LBFS_OK ? (double)t / reps : 0.0;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

// a candidate replaces the best so far (initially the default) only when it is faster
// by more than the run-to-run spread of such timings (2 %)
bool clearly_faster(double t, double best) { return t < 0.98 * best; }

// Time candidates 0..n-1 with time_one(k, &ms) in two passes, forward then backward, and
// keep each candidate's shorter time: a drifting clock (the GPU's, rising after the host
// copies that restore the state) then favours neither end of the list. Returns the
// index of the fastest, the default `def` unless a candidate is clearly faster.
template <typename F>
int time_candidates(int n, int def, double* t, int& rc, F&& time_one)
{
    for (int pass = 0; pass < 2; pass++)
        for (int j = 0; j < n && rc == LBFS_OK; j++) {
            const int k = pass ? n - 1 - j : j;
            double ms = 0.0;
            rc = time_one(k, &ms);
            if (rc == LBFS_OK) t[k] = pass ? std::min(t[k], ms) : ms;
        }
    int best = def;
    for (int k = 0; k < n && rc == LBFS_OK; k++)
        if (k != def && clearly_faster(t[k], t[best])) best = k;
    return best;
}

// stand-in for the three Runge-Kutta stages of a step: stage 1, then stage 2 twice
// (stage 3 writes the state; its cost follows stage 2's, which reads as many fields).
// Both write only the stage fields W1 and W2, so timing them leaves the state as it is.
hipError_t stage_pair(Exec& E)
{
    hipError_t e = exec_stage(E, 1);
    if (e == hipSuccess) e = exec_stage(E, 2);
    return e == hipSuccess ? exec_stage(E, 2) : e;
}

// the potential of an instance: saved to / restored from the stage-2 field He (free
// between steps; the stage timing that writes it comes first)
hipError_t copy_phi(lbfs_solver* s, bool save)
{
    void* phi = s->field(s->phi_field());
    void* keep = s->field(10);
    return hipMemcpyAsync(save ? keep : phi, save ? phi : keep, s->L.field_bytes, hipMemcpyDeviceToDevice,
                          s->stream);
}

}  // namespace

extern "C" {

int lbfs_tile_shape(int32_t kind, int32_t precision, int32_t index, int32_t* tx, int32_t* ty, int32_t* threads,
                    int32_t* flags)
{
    if (precision != LBFS_FP32 && precision != LBFS_FP64) return LBFS_E_INVAL;
    const int n = kind == 0 ? NSTAGE_SHAPES : kind == 1 ? NMAG_SHAPES : -1;
    if (n < 0) return LBFS_E_INVAL;
    if (index < 0) return n;
    if (kind == 1 && index == n) {   // the sweeps inside stage 1, on its tiles
        if (tx) *tx = 0;
        if (ty) *ty = 0;
        if (threads) *threads = 0;
        if (flags) *flags = 2;
        return LBFS_OK;
    }
    if (index >= n) return LBFS_E_INVAL;
    const TileShape S = kind == 0 ? stage_shape(precision == LBFS_FP64, index) : MAG_SHAPES[index];
    if (tx) *tx = S.tx;
    if (ty) *ty = S.ty;
    if (threads) *threads = S.nt;
    if (flags) *flags = S.early ? 1 : 0;
    return LBFS_OK;
}

int lbfs_set_tile_shapes(lbfs_solver* s, int32_t stage_shape_idx, int32_t mag_shape_idx)
{
    if (!s || s->batched) return LBFS_E_STATE;
    if (stage_shape_idx < 0 || stage_shape_idx >= NSTAGE_SHAPES || mag_shape_idx < 0 || mag_shape_idx > NMAG_SHAPES)
        return LBFS_E_INVAL;
    const bool mag_changed = mag_shape_idx != NMAG_SHAPES && mag_shape_idx != s->E.mag_shape;
    int rc = apply_shapes(s, stage_shape_idx, mag_shape_idx);
    if (rc != LBFS_OK) return rc;
    // residual partials of the current potential on the new magnetic tiles
    if (mag_changed) {
        HIPCHK(exec_mag(s->E, 0, 1.0, 1));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    return LBFS_OK;
}

int lbfs_tile_shapes_in_use(const lbfs_solver* s, int32_t* stage_shape_idx, int32_t* mag_shape_idx)
{
    if (!s) return LBFS_E_STATE;
    if (stage_shape_idx) *stage_shape_idx = s->E.stage_shape;
    if (mag_shape_idx) *mag_shape_idx = s->E.fused ? NMAG_SHAPES : s->E.mag_shape;
    return LBFS_OK;
}

int lbfs_autotune(lbfs_solver* s, int32_t reps, int32_t* chosen, double* ms)
{
    if (!s || s->batched) return LBFS_E_STATE;
    if (reps < 1 || reps > 10000) return LBFS_E_INVAL;
    Exec& E = s->E;
    double t[2 * LBFS_MAX_SHAPES] = {0};
    const int phase0 = E.phase;
    const int mag0 = E.mag_shape;
    // Candidates are timed on whole time steps (direct launches), each from the same
    // state: a host snapshot in the checkpoint format, loaded again before every
    // candidate and at the end. (Timing stage 1 and stage 2 alone, which leave the
    // state as it is, ranked tile shapes a few percent differently from whole steps.)
    std::vector<char> snap(lbfs_checkpoint_bytes(s));
    int rc = lbfs_save_state(s, snap.data(), snap.size());
    auto restore = [&]() {
        E.phase = phase0;
        return lbfs_load_state(s, snap.data(), snap.size());
    };
    auto time_steps = [&](double* out) {
        int r = restore();
        if (r == LBFS_OK) r = time_launches(E.stream, reps, [&] { return exec_enqueue_step(E); }, out);
        return r;
    };
    // stage shapes with the current magnetic shape, then magnetic shapes with the best
    // stage shape
    const int best_s = time_candidates(NSTAGE_SHAPES, default_stage_shape(s->f64(), (size_t)s->p.nx * s->p.ny), t,
                                       rc, [&](int k, double* ms) {
        int r = apply_shapes(s, k, mag0);
        return r == LBFS_OK ? time_steps(ms) : r;
    });
    const int best_m = time_candidates(NMAG_SHAPES, 0, t + LBFS_MAX_SHAPES, rc, [&](int k, double* ms) {
        int r = apply_shapes(s, best_s, k);
        return r == LBFS_OK ? time_steps(ms) : r;
    });
    // the sweeps inside stage 1 (its tiles plus a wider halo, one launch less per step)
    bool fuse = false;
    if (rc == LBFS_OK && fusable(s->p)) {
        double tf = 0.0;
        rc = apply_shapes(s, best_s, NMAG_SHAPES);
        if (rc == LBFS_OK) rc = time_steps(&tf);
        if (rc == LBFS_OK) {
            t[LBFS_MAX_SHAPES + NMAG_SHAPES] = tf - t[LBFS_MAX_SHAPES + best_m];
            fuse = clearly_faster(tf, t[LBFS_MAX_SHAPES + best_m]);
        }
    }
    // the state as it was, the fastest shapes, and the residual partials of the restored
    // potential on them (a sweep-free launch: a copy of the potential)
    const int rr = restore();
    if (rc == LBFS_OK) rc = rr;
    if (rc == LBFS_OK) rc = apply_shapes(s, best_s, best_m);
    if (rc == LBFS_OK && fuse) rc = apply_shapes(s, best_s, NMAG_SHAPES);
    if (rc == LBFS_OK && (HIPFAIL(exec_mag(E, 0, 1.0, 1)) || HIPFAIL(hipStreamSynchronize(E.stream))))
        rc = LBFS_E_DEVICE;
    s->stepped_since_observe = true;
    if (rc != LBFS_OK) return rc;
    if (chosen) {
        chosen[0] = best_s;
        chosen[1] = fuse ? NMAG_SHAPES : best_m;
    }
    if (ms)
        for (int k = 0; k < 2 * LBFS_MAX_SHAPES; k++) ms[k] = t[k];
    return LBFS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches

namespace {

// first-fit allocator over [0, size) in ALIGN units, coalescing on free
struct Arena {
    std::map<size_t, size_t> free_;   // offset -> length
    void reset(size_t size)
    {
        free_.clear();
        if (size > 0) free_[0] = size;
    }
    bool alloc(size_t len, size_t* off)
    {
        len = align_up(len, ALIGN);
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= len) {
                *off = it->first;
                const size_t rest = it->second - len, at = it->first + len;
                free_.erase(it);
                if (rest > 0) free_[at] = rest;
                return true;
            }
        return false;
    }
    void release(size_t off, size_t len)
    {
        len = align_up(len, ALIGN);
        auto it = free_.emplace(off, len).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest() const
    {
        size_t m = 0;
        for (const auto& kv : free_) m = kv.second > m ? kv.second : m;
        return m;
    }
};

struct Slot {
    lbfs_solver* s = nullptr;
    size_t off = 0, bytes = 0;
};

}  // namespace

struct lbfs_batch {
    int32_t max_slots = 0, precision = 0, sweeps = 0;
    int stage_shape = 0, mag_shape = 0;   // tile shapes of every instance
    bool shapes_given = false;            // set by lbfs_batch_set_tile_shapes or the autotuner
    double omega = 1.0;
    char* base = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    Arena arena;
    std::vector<Slot> slots;
    // metadata block: DevInst[max_slots] | results[max_slots][NRES] | stage tiles | magnetic tiles
    size_t meta_off = 0, meta_bytes = 0;
    int cap_stage = 0, cap_mag = 0;
    std::vector<int32_t> compact;   // compact instance index -> slot
    double* hres = nullptr;         // pinned [max_slots][NRES]
    bool dirty = true, stepped_since_observe = true;
    Exec E;
    DevInst* meta_inst() const { return reinterpret_cast<DevInst*>(base + meta_off); }
    double* meta_res() const
    {
        return reinterpret_cast<double*>(base + meta_off + align_up(sizeof(DevInst) * max_slots, ALIGN));
    }
    Tile* meta_stage() const
    {
        return reinterpret_cast<Tile*>(reinterpret_cast<char*>(meta_res()) +
                                       align_up(sizeof(double) * NRES * max_slots, ALIGN));
    }
    Tile* meta_mag() const
    {
        return reinterpret_cast<Tile*>(reinterpret_cast<char*>(meta_stage()) +
                                       align_up(sizeof(Tile) * cap_stage, ALIGN));
    }
};

namespace {

size_t meta_size(int max_slots, int cap_stage, int cap_mag)
{
    return align_up(sizeof(DevInst) * max_slots, ALIGN) + align_up(sizeof(double) * NRES * max_slots, ALIGN) +
           align_up(sizeof(Tile) * cap_stage, ALIGN) + align_up(sizeof(Tile) * cap_mag, ALIGN);
}

// make room in the metadata block for need_stage / need_mag tiles (grows by half
// again, so admissions rarely move it); the old block is released after the stream
// has drained (a captured graph may still read it)
int batch_reserve(lbfs_batch* b, int need_stage, int need_mag)
{
    if (need_stage <= b->cap_stage && need_mag <= b->cap_mag && b->meta_bytes > 0) return LBFS_OK;
    const int cs = need_stage > b->cap_stage ? need_stage + need_stage / 2 : b->cap_stage;
    const int cm = need_mag > b->cap_mag ? need_mag + need_mag / 2 : b->cap_mag;
    const size_t nb = meta_size(b->max_slots, cs, cm);
    size_t off = 0;
    if (!b->arena.alloc(nb, &off)) {
        // retry at the exact size
        const size_t nb2 = meta_size(b->max_slots, need_stage, need_mag);
        if (!b->arena.alloc(nb2, &off)) return LBFS_E_NOMEM;
        if (HIPFAIL(hipStreamSynchronize(b->stream))) {
            b->arena.release(off, nb2);
            return LBFS_E_DEVICE;
        }
        if (b->meta_bytes) b->arena.release(b->meta_off, b->meta_bytes);
        b->meta_off = off;
        b->meta_bytes = nb2;
        b->cap_stage = need_stage;
        b->cap_mag = need_mag;
        b->dirty = true;
        return LBFS_OK;
    }
    if (HIPFAIL(hipStreamSynchronize(b->stream))) {
        b->arena.release(off, nb);
        return LBFS_E_DEVICE;
    }
    if (b->meta_bytes) b->arena.release(b->meta_off, b->meta_bytes);
    b->meta_off = off;
    b->meta_bytes = nb;
    b->cap_stage = cs;
    b->cap_mag = cm;
    b->dirty = true;
    return LBFS_OK;
}

// rebuild the descriptors and tile lists of the live instances and drop the graphs
int batch_rebuild(lbfs_batch* b)
{
    if (!b->dirty) return LBFS_OK;
    if (HIPFAIL(hipStreamSynchronize(b->stream))) return LBFS_E_DEVICE;
    exec_drop_graphs(b->E);
    b->compact.clear();
    std::vector<DevInst> insts;
    std::vector<Tile> ts, tm;
    const TileShape SS = stage_shape(b->precision == LBFS_FP64, b->stage_shape), MS = MAG_SHAPES[b->mag_shape];
    for (int k = 0; k < b->max_slots; k++) {
        lbfs_solver* s = b->slots[k].s;
        if (!s) continue;
        const int c = (int)b->compact.size();
        b->compact.push_back(k);
        DevInst I = s->hinst;
        I.result = b->meta_res() + (size_t)NRES * c;
        I.ntile_stage = count_tiles(s->p.nx, s->p.ny, SS);
        I.ntile_mag = count_tiles(s->p.nx, s->p.ny, MS);
        insts.push_back(I);
        append_tiles(ts, c, s->p.nx, s->p.ny, SS);
        append_tiles(tm, c, s->p.nx, s->p.ny, MS, true);
    }
    if ((int)ts.size() > b->cap_stage || (int)tm.size() > b->cap_mag) return LBFS_E_STATE;
    if (!insts.empty()) {
        HIPCHK(hipMemcpyAsync(b->meta_inst(), insts.data(), sizeof(DevInst) * insts.size(), hipMemcpyHostToDevice,
                              b->stream));
        HIPCHK(hipMemcpyAsync(b->meta_stage(), ts.data(), sizeof(Tile) * ts.size(), hipMemcpyHostToDevice, b->stream));
        HIPCHK(hipMemcpyAsync(b->meta_mag(), tm.data(), sizeof(Tile) * tm.size(), hipMemcpyHostToDevice, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
    }
    Exec& E = b->E;
    E.mu_ready = false;   // (a new member's kf[0] holds no permeability yet)
    E.dinst = b->meta_inst();
    E.ninst = (int)insts.size();
    E.tiles_stage = b->meta_stage();
    E.nstage = (int)ts.size();
    E.tiles_mag = b->meta_mag();
    E.nmag = (int)tm.size();
    E.stage_shape = b->stage_shape;
    E.mag_shape = b->mag_shape;
    b->dirty = false;
    return LBFS_OK;
}

void batch_after_step(lbfs_batch* b)
{
    for (int k = 0; k < b->max_slots; k++) {
        lbfs_solver* s = b->slots[k].s;
        if (!s) continue;
        s->t += s->p.dt;
        s->step += 1;
        s->E.phase = b->E.phase;
        s->stepped_since_observe = true;
    }
    b->stepped_since_observe = true;
}

}  // namespace

extern "C" {

size_t lbfs_batch_instance_bytes(const lbfs_params* p)
{
    if (validate(p) != LBFS_OK) return 0;
    return align_up(make_layout(p).total, ALIGN);
}

int lbfs_batch_create(int32_t max_slots, int32_t precision, int32_t sweeps, double sor_omega, void* dev_buf,
                      size_t bytes, void* stream, lbfs_batch** out)
{
    if (!out) return LBFS_E_INVAL;
    *out = nullptr;
    if (max_slots < 1 || max_slots > (1 << 16) || !dev_buf) return LBFS_E_INVAL;
    if (precision != LBFS_FP32 && precision != LBFS_FP64) return LBFS_E_INVAL;
    if (sweeps < 0 || sweeps > 1000 || !(sor_omega > 0.0 && sor_omega < 2.0)) return LBFS_E_INVAL;
    lbfs_batch* b = new (std::nothrow) lbfs_batch();
    if (!b) return LBFS_E_NOMEM;
    b->max_slots = max_slots;
    b->precision = precision;
    b->sweeps = sweeps;
    b->omega = sor_omega;
    char* base = reinterpret_cast<char*>(align_up(reinterpret_cast<uintptr_t>(dev_buf), ALIGN));
    const size_t lost = (size_t)(base - static_cast<char*>(dev_buf));
    b->base = base;
    b->bytes = bytes > lost ? (bytes - lost) / ALIGN * ALIGN : 0;
    b->arena.reset(b->bytes);
    b->stream = static_cast<hipStream_t>(stream);
    b->slots.assign(max_slots, Slot{});
    Exec& E = b->E;
    E.f64 = precision == LBFS_FP64;
    E.sweeps = sweeps;
    E.omega = sor_omega;
    E.stream = b->stream;
    const char* ng = std::getenv("LBFS_NO_GRAPH");
    E.use_graph = b->stream != nullptr && !(ng && ng[0] == '1');
    exec_set_graph_steps(E, graph_steps_setting());
    if (HIPFAIL(hipHostMalloc(&b->hres, sizeof(double) * NRES * max_slots, hipHostMallocDefault))) {
        delete b;
        return LBFS_E_DEVICE;
    }
    const int rc = batch_reserve(b, 0, 0);
    if (rc != LBFS_OK) {
        lbfs_batch_destroy(b);
        return rc;
    }
    *out = b;
    return LBFS_OK;
}

// a batch whose shapes were not given takes the stage and magnetic shapes of a step
// over its total cells (with many instances the tiles fill the GPU as one large grid's do),
// stepping down to smaller tiles while the shape's tiles would cover more than 15%
// beyond the instances' cells (edges that are no multiple of the tile); an instance of
// nx x ny about to be admitted counts too
static int batch_follow_size(lbfs_batch* b, int nx = 0, int ny = 0)
{
    if (b->shapes_given) return LBFS_OK;
    size_t cells = (size_t)nx * ny;
    for (const Slot& q : b->slots)
        if (q.s) cells += (size_t)q.s->p.nx * q.s->p.ny;
    auto covered = [&](int k) {
        const TileShape S = MAG_SHAPES[k];
        size_t a = nx > 0 ? (size_t)count_tiles(nx, ny, S) * S.tx * S.ty : 0;
        for (const Slot& q : b->slots)
            if (q.s) a += (size_t)count_tiles(q.s->p.nx, q.s->p.ny, S) * S.tx * S.ty;
        return a;
    };
    int m = default_mag_shape(cells);   // 1 (64 x 32), 2 (64 x 16) or 0 (32 x 8)
    while (m != 0 && (double)covered(m) > 1.15 * (double)cells) m = m == 1 ? 2 : 0;
    const int st = default_stage_shape(b->precision == LBFS_FP64, cells);
    if (m == b->mag_shape && st == b->stage_shape) return LBFS_OK;
    const int rc = lbfs_batch_set_tile_shapes(b, st, m);
    b->shapes_given = false;
    return rc;
}

int lbfs_batch_admit(lbfs_batch* b, const lbfs_params* p, int32_t* slot_out)
{
    if (!b) return LBFS_E_STATE;
    if (!p || !slot_out) return LBFS_E_INVAL;
    const int v = validate(p);
    if (v != LBFS_OK) return v;
    if (p->precision != b->precision || p->sweeps != b->sweeps || p->sor_omega != b->omega ||
        p->mag_method != LBFS_MAG_SWEEPS || p->mag_max_iters != 0)
        return LBFS_E_INVAL;
    int slot = -1;
    for (int k = 0; k < b->max_slots && slot < 0; k++)
        if (!b->slots[k].s) slot = k;
    if (slot < 0) return LBFS_E_NOMEM;
    // room for the tiles of every instance under any candidate shape
    const Layout L = make_layout(p);
    int ns = L.cap_stage, nm = L.cap_mag;
    for (const Slot& q : b->slots)
        if (q.s) {
            ns += q.s->L.cap_stage;
            nm += q.s->L.cap_mag;
        }
    int rc = batch_reserve(b, ns, nm);
    if (rc != LBFS_OK) return rc;
    // the shapes with the new instance counted, before it takes them
    rc = batch_follow_size(b, p->nx, p->ny);
    if (rc != LBFS_OK) return rc;
    const size_t need = align_up(L.total, ALIGN);
    size_t off = 0;
    if (!b->arena.alloc(need, &off)) return LBFS_E_NOMEM;
    lbfs_solver* s = nullptr;
    rc = init_solver(p, b->base + off, need, b->stream, &s);
    if (rc != LBFS_OK) {
        b->arena.release(off, need);
        return rc;
    }
    // the member's own tile lists take the batch's shapes, and its residual partials are
    // recomputed on them (a sweep-free magnetic launch: a copy of the potential)
    if (s->E.stage_shape != b->stage_shape || s->E.mag_shape != b->mag_shape) {
        if (apply_shapes(s, b->stage_shape, b->mag_shape) != LBFS_OK || HIPFAIL(exec_mag(s->E, 0, 1.0, 1))) {
            destroy_solver(s);
            b->arena.release(off, need);
            return LBFS_E_DEVICE;
        }
    }
    // bring the potential into the batch's current buffer
    if (s->E.phase != b->E.phase) {
        const int from = s->phi_field();
        s->E.phase = b->E.phase;
        if (HIPFAIL(hipMemcpyAsync(s->field(s->phi_field()), s->field(from), s->L.field_bytes,
                                   hipMemcpyDeviceToDevice, b->stream)) ||
            HIPFAIL(hipStreamSynchronize(b->stream))) {
            destroy_solver(s);
            b->arena.release(off, need);
            return LBFS_E_DEVICE;
        }
    }
    s->batched = true;
    s->owner_stale = &b->stepped_since_observe;
    s->owner_mu = &b->E.mu_ready;
    b->slots[slot] = Slot{s, off, need};
    b->dirty = true;
    b->stepped_since_observe = true;
    *slot_out = slot;
    return LBFS_OK;
}

int lbfs_batch_retire(lbfs_batch* b, int32_t slot)
{
    if (!b) return LBFS_E_STATE;
    if (slot < 0 || slot >= b->max_slots) return LBFS_E_INVAL;
    Slot& q = b->slots[slot];
    if (!q.s) return LBFS_E_STATE;
    HIPCHK(hipStreamSynchronize(b->stream));
    destroy_solver(q.s);
    b->arena.release(q.off, q.bytes);
    q = Slot{};
    b->dirty = true;
    b->stepped_since_observe = true;
    return batch_follow_size(b);
}

int lbfs_batch_step(lbfs_batch* b, int32_t nsteps)
{
    if (!b) return LBFS_E_STATE;
    if (nsteps < 0) return LBFS_E_INVAL;
    const int rc = batch_rebuild(b);
    if (rc != LBFS_OK) return rc;
    if (b->E.ninst == 0) return LBFS_OK;
    for (int n = 0; n < nsteps;) {
        const int k = exec_run_steps(b->E, nsteps - n);
        if (k == 0) return LBFS_E_DEVICE;
        for (int q = 0; q < k; q++) batch_after_step(b);
        n += k;
    }
    return LBFS_OK;
}

int lbfs_batch_prepare(lbfs_batch* b)
{
    if (!b) return LBFS_E_STATE;
    const int rc = batch_rebuild(b);
    if (rc != LBFS_OK) return rc;
    HIPCHK(exec_prepare(b->E));
    return LBFS_OK;
}

int lbfs_batch_step_profiled_start(lbfs_batch* b, int32_t nsteps, int32_t sample_every)
{
    if (!b) return LBFS_E_STATE;
    if (nsteps < 0 || sample_every < 1) return LBFS_E_INVAL;
    if (b->E.prof_pending) return LBFS_E_STATE;
    const int rc = batch_rebuild(b);
    if (rc != LBFS_OK) return rc;
    if (b->E.ninst == 0) nsteps = 0;
    return exec_profiled_start(b->E, nsteps, sample_every, [&] { batch_after_step(b); });
}

int lbfs_batch_profile_result(lbfs_batch* b, double* kernel_ms, int32_t* launches)
{
    if (!b) return LBFS_E_STATE;
    if (!kernel_ms || !launches) return LBFS_E_INVAL;
    return exec_profiled_result(b->E, kernel_ms, launches);
}

int lbfs_batch_step_profiled(lbfs_batch* b, int32_t nsteps, int32_t sample_every, double* kernel_ms,
                             int32_t* launches)
{
    if (!b) return LBFS_E_STATE;
    if (nsteps < 0 || sample_every < 1 || !kernel_ms || !launches) return LBFS_E_INVAL;
    const int rc = lbfs_batch_step_profiled_start(b, nsteps, sample_every);
    return rc == LBFS_OK ? lbfs_batch_profile_result(b, kernel_ms, launches) : rc;
}

int lbfs_batch_observe(lbfs_batch* b, lbfs_observables* out, uint8_t* live)
{
    if (!b) return LBFS_E_STATE;
    if (!out || !live) return LBFS_E_INVAL;
    int rc = batch_rebuild(b);
    if (rc != LBFS_OK) return rc;
    const int n = b->E.ninst;
    if (b->stepped_since_observe && n > 0) {
        HIPCHK(exec_state_partials(b->E));
        HIPCHK(launch_reduce(b->E.dinst, n, b->stream));
        HIPCHK(hipMemcpyAsync(b->hres, b->meta_res(), sizeof(double) * NRES * n, hipMemcpyDeviceToHost, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
        b->stepped_since_observe = false;
    }
    rc = LBFS_OK;
    for (int k = 0; k < b->max_slots; k++) {
        live[k] = 0;
        std::memset(&out[k], 0, sizeof out[k]);
    }
    for (int c = 0; c < n; c++) {
        const int k = b->compact[c];
        lbfs_solver* s = b->slots[k].s;
        live[k] = 1;
        if (fill_observables(s->p, s->t, s->step, s->vol0, b->hres + (size_t)NRES * c, &out[k]) != LBFS_OK)
            rc = LBFS_E_NONFINITE;
    }
    return rc;
}

int lbfs_batch_slot(lbfs_batch* b, int32_t slot, lbfs_solver** out)
{
    if (!b) return LBFS_E_STATE;
    if (!out || slot < 0 || slot >= b->max_slots) return LBFS_E_INVAL;
    *out = b->slots[slot].s;
    return *out ? LBFS_OK : LBFS_E_STATE;
}

int lbfs_batch_info(lbfs_batch* b, int32_t* live, int64_t* cells, size_t* largest_free)
{
    if (!b) return LBFS_E_STATE;
    int32_t n = 0;
    int64_t c = 0;
    for (const Slot& q : b->slots)
        if (q.s) {
            n++;
            c += (int64_t)q.s->p.nx * q.s->p.ny;
        }
    if (live) *live = n;
    if (cells) *cells = c;
    if (largest_free) *largest_free = b->arena.largest();
    return LBFS_OK;
}

// residual partials of every member's current potential on the batch's magnetic tiles
static int batch_refresh_residual(lbfs_batch* b)
{
    HIPCHK(exec_mag(b->E, 0, 1.0, 1));
    HIPCHK(hipStreamSynchronize(b->stream));
    for (Slot& q : b->slots)
        if (q.s) q.s->E.phase = b->E.phase;
    b->stepped_since_observe = true;
    return LBFS_OK;
}

int lbfs_batch_set_tile_shapes(lbfs_batch* b, int32_t stage_shape_idx, int32_t mag_shape_idx)
{
    if (!b) return LBFS_E_STATE;
    if (stage_shape_idx < 0 || stage_shape_idx >= NSTAGE_SHAPES || mag_shape_idx < 0 || mag_shape_idx >= NMAG_SHAPES)
        return LBFS_E_INVAL;
    b->shapes_given = true;
    HIPCHK(hipStreamSynchronize(b->stream));
    const bool mag_changed = mag_shape_idx != b->mag_shape;
    b->stage_shape = stage_shape_idx;
    b->mag_shape = mag_shape_idx;
    for (Slot& q : b->slots)   // the members' own lists (used through borrowed handles)
        if (q.s) {
            const int rc = apply_shapes(q.s, stage_shape_idx, mag_shape_idx);
            if (rc != LBFS_OK) return rc;
        }
    b->dirty = true;
    b->stepped_since_observe = true;
    int rc = batch_rebuild(b);
    if (rc == LBFS_OK && mag_changed && b->E.ninst > 0) rc = batch_refresh_residual(b);
    return rc;
}

int lbfs_batch_autotune(lbfs_batch* b, int32_t reps, int32_t* chosen, double* ms)
{
    if (!b) return LBFS_E_STATE;
    if (reps < 1 || reps > 10000) return LBFS_E_INVAL;
    int rc = batch_rebuild(b);
    if (rc != LBFS_OK) return rc;
    double t[2 * LBFS_MAX_SHAPES] = {0};
    int best_s = b->stage_shape, best_m = b->mag_shape;
    Exec& E = b->E;
    if (E.ninst > 0) {
        // whole steps of every instance from host snapshots, as in lbfs_autotune
        const int phase0 = E.phase;
        size_t cells = 0;
        for (const Slot& q : b->slots)
            if (q.s) cells += (size_t)q.s->p.nx * q.s->p.ny;
        std::vector<std::vector<char>> snap(b->slots.size());
        for (size_t i = 0; i < b->slots.size() && rc == LBFS_OK; i++)
            if (lbfs_solver* q = b->slots[i].s) {
                snap[i].resize(lbfs_checkpoint_bytes(q));
                rc = lbfs_save_state(q, snap[i].data(), snap[i].size());
            }
        auto restore = [&]() {
            E.phase = phase0;
            int r = LBFS_OK;
            for (size_t i = 0; i < b->slots.size() && r == LBFS_OK; i++)
                if (lbfs_solver* q = b->slots[i].s) {
                    q->E.phase = phase0;
                    r = lbfs_load_state(q, snap[i].data(), snap[i].size());
                }
            return r;
        };
        auto time_steps = [&](double* out) {
            int r = batch_rebuild(b);
            if (r == LBFS_OK) r = restore();
            if (r == LBFS_OK) r = time_launches(E.stream, reps, [&] { return exec_enqueue_step(E); }, out);
            return r;
        };
        best_s = time_candidates(NSTAGE_SHAPES, default_stage_shape(b->precision == LBFS_FP64, cells), t, rc,
                                 [&](int k, double* ms) {
            b->stage_shape = k;
            b->dirty = true;
            return time_steps(ms);
        });
        b->stage_shape = best_s;
        best_m = time_candidates(NMAG_SHAPES, 0, t + LBFS_MAX_SHAPES, rc, [&](int k, double* ms) {
            b->mag_shape = k;
            b->dirty = true;
            return time_steps(ms);
        });
        const int rr = restore();
        if (rc == LBFS_OK) rc = rr;
        b->stepped_since_observe = true;
        if (rc != LBFS_OK) return rc;
        rc = lbfs_batch_set_tile_shapes(b, best_s, best_m);
        if (rc == LBFS_OK) rc = batch_refresh_residual(b);
        if (rc != LBFS_OK) return rc;
    }
    if (chosen) {
        chosen[0] = best_s;
        chosen[1] = best_m;
    }
    if (ms)
        for (int k = 0; k < 2 * LBFS_MAX_SHAPES; k++) ms[k] = t[k];
    return LBFS_OK;
}

int lbfs_batch_tile_shapes_in_use(const lbfs_batch* b, int32_t* stage_shape_idx, int32_t* mag_shape_idx)
{
    if (!b) return LBFS_E_STATE;
    if (stage_shape_idx) *stage_shape_idx = b->stage_shape;
    if (mag_shape_idx) *mag_shape_idx = b->mag_shape;
    return LBFS_OK;
}

void lbfs_batch_destroy(lbfs_batch* b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    exec_release(b->E);
    for (Slot& q : b->slots)
        if (q.s) destroy_solver(q.s);
    if (b->hres) (void)hipHostFree(b->hres);
    delete b;
}

}  // extern "C"

// lbfs_internal.hpp -- structures shared by the host ABI and the gfx950 kernels.
//
// Every kernel works on a list of tiles; a tile names the instance it belongs to and
// its origin. One solver is a list of one instance; a batch is the same kernels over
// the tiles of many instances, so a batched instance computes exactly what it
// computes alone.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbfs {

// Tile shapes (cells) and workgroup sizes. The kernels loop over their tile plus halo
// and over its faces, so any shape works; these are the candidates the autotuner times
// (index 0, the default but for FP64 grids above 512^2, was among the fastest on 1024^2
// grids and on batches).
// Stage kernels stage the tile plus a 3-cell halo.
struct TileShape {
    int tx, ty, nt;
    int early = 0;   // stage kernels: stage 0/1 load the owned cell's values before the halo
};
// Small workgroups: with the stage kernels' register use (69 VGPRs in FP32, 128 to 156 in
// FP64) only a few waves fit per SIMD, and several small workgroups per CU hide each
// other's barrier and LDS waits better than one large one, although small tiles
// recompute more halo cells (2.6x for 10 x 10) and faces (2.2 per cell).
// The face phase gives each wave faces of one axis: the x-faces ((TX+1) TY) and the
// y-faces (TX (TY+1)) are each rounded up to whole waves, so 10 x 10 (110 + 110 faces on
// four waves, a 256-cell halo region in one round, 22 KB of LDS in FP32: seven
// workgroups and seven waves per SIMD) keeps the lanes busy: a whole step on a 1024^2
// grid takes 126 us against 137 us with 10 x 8 (4 face waves for 178 faces). In FP64 the
// 10 x 10 tile needs 44 KB of LDS (three workgroups per CU); 10 x 8 needs 38 KB and
// 12 x 7 40 KB, so four fit, and the stage kernel is held to 128 VGPRs for four waves
// per SIMD. 10 x 8 is the FP64 default up to 512^2 cells, 12 x 7 above (a whole step on
// 1024^2: 258 us against 265 us for 10 x 8 and 274 us for 12 x 8; on 256^2 10 x 8 is
// ahead by 1.5%). Loading the owned cell's values early
// hides their latency but holds registers through the face phase; whether that costs a
// wave per SIMD depends on the shape, so both are candidates.
constexpr int NSTAGE_SHAPES = 7;
constexpr TileShape STAGE_SHAPES_F32[NSTAGE_SHAPES] = {
    {10, 10, 256, 0}, {10, 8, 256, 0}, {12, 7, 256, 1}, {12, 7, 256, 0}, {12, 8, 256, 0}, {8, 8, 192, 0},
    {8, 12, 256, 0}};
constexpr TileShape STAGE_SHAPES_F64[NSTAGE_SHAPES] = {
    {10, 8, 256, 0}, {10, 10, 256, 0}, {12, 8, 256, 0}, {8, 8, 256, 0}, {12, 7, 256, 0}, {8, 7, 192, 0},
    {8, 8, 192, 0}};
// fused magnetic kernel: interior tile shapes; one launch does up to MAG_KMAX sweeps
// (LDS halo 2*MAG_KMAX, one ring more in a launch that computes the residual). Without
// autotuning, grids above 512 x 512 use shape 1 (a larger tile recomputes fewer halo
// cells: 1.9x for 64 x 32 against 2.5x for 64 x 16).
constexpr int MAG_KMAX = 4;
constexpr int NMAG_SHAPES = 5;
constexpr TileShape MAG_SHAPES[NMAG_SHAPES] = {{32, 8, 704}, {64, 32, 1024}, {64, 16, 1024}, {64, 8, 1024},
                                               {128, 16, 1024}};
// The magnetic LBFS pseudo-time solve runs on the same tiles: one launch does up to
// RK_KMAX pseudo-steps of three stages each (LDS halo 3*RK_KMAX+1).
constexpr int RK_KMAX = 4;

constexpr TileShape stage_shape(bool f64, int k) { return f64 ? STAGE_SHAPES_F64[k] : STAGE_SHAPES_F32[k]; }
// pointwise kernels (init, derived fields): one thread per cell
constexpr int PT_TX = 64, PT_TY = 4;

// per-tile partial sums of the observables of a state (FP64)
enum { PART_CT = 0, PART_CTFL, PART_FS, PART_UMAX, PART_NONFINITE, PART_UDROP, PART_HEIGHT,
       PART_HEAT, PART_MX, PART_MY, PART_MXX, PART_MYY, PART_MXY, PART_SOLIDH, NPART };
// per-instance results written by the reduction (FP64)
enum { RES_CT = 0, RES_CTFL, RES_FS, RES_UMAX, RES_NONFINITE, RES_UDROP, RES_HEIGHT, RES_HEAT,
       RES_MX, RES_MY, RES_MXX, RES_MYY, RES_MXY, RES_SOLIDH, RES_MAGR2, NRES };

struct Tile {
    int32_t inst;    // instance index
    int32_t x0, y0;  // origin (cells)
    int32_t idx;     // row-major tile index inside its instance (partials slot)
};

// Position k of an instance's tile list -> tile (tx, ty) of its ntx x nty tiles of tw x
// th cells. Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2, and the kernels hand each XCD one contiguous eighth of the list (xcd_tile). This
// order lists the tiles as 8 rectangular blocks, row-major inside each, so that an
// eighth is a compact rectangle: the halo cells it re-reads across XCD boundaries lie
// along its perimeter, shorter than that of a full-width strip of the same area (the
// row-major order). The blocks split the grid into
// bx x (8 / bx), bx in {1, 2, 4, 8}, the most square in cells; a grid of fewer tiles
// than that is listed row-major.
__host__ __device__ inline void tile_at(int k, int ntx, int nty, int tw, int th, int& tx, int& ty)
{
    int bx = 0;
    long best = 0;
    for (int b = 1; b <= 8; b *= 2) {
        const int c = 8 / b;
        if (b > ntx || c > nty) continue;
        const long per = (long)ntx * tw / b + (long)nty * th / c;   // block half-perimeter (cells)
        if (bx == 0 || per < best) {
            bx = b;
            best = per;
        }
    }
    if (bx == 0) {
        tx = k % ntx;
        ty = k / ntx;
        return;
    }
    const int by = 8 / bx;
    for (int j = 0; j < by; j++) {
        const int y0 = j * nty / by, y1 = (j + 1) * nty / by;
        for (int i = 0; i < bx; i++) {
            const int x0 = i * ntx / bx, x1 = (i + 1) * ntx / bx;
            const int n = (x1 - x0) * (y1 - y0);
            if (k < n) {
                tx = x0 + k % (x1 - x0);
                ty = y0 + k / (x1 - x0);
                return;
            }
            k -= n;
        }
    }
    tx = ty = 0;   // (k beyond the grid: not reached for k < ntx nty)
}

// Parameters of one instance in one precision, with the derived constants the kernels
// need precomputed on the host: the kernels read them as uniform scalars (no per-thread
// conversion from FP64, no per-thread division of constants).
template <typename T>
struct Coef {
    T rho[3], mu[3], lam[3], cp[3], chi[3];   // [solid, liquid, gas] (Eq. 11)
    T tval[4];                                // fixed wall temperatures
    T wet[4];                                 // (4 / xi) cos(contact angle) per wall, 0 at 90 degrees
    T latent, tm, tl, dx, dt, cpref, qg, tau_g, beta, kappa, mu0, h0x, h0y, vc;   // tm, tl: Ts, Tl
    T grav[2];
    T idx;      // 1 / dx
    T inv2dx;   // 1 / (2 dx)
    T idx2;     // 1 / dx^2
    T i_halfdx; // 2 / dx
    T idt;      // 1 / dt
    T tauf_k;   // 3 / delta_t:           tau_f = 1/2 + (mu / rho) tauf_k
    T tauh_k;   // 3 / (Cp,ref delta_t):  tau_h = 1/2 + (lambda / rho) tauh_k
    T mag_kdt;  // D dtau / dx^2 of the magnetic pseudo-time solve
};

// Per-instance descriptor, resident in device memory. Field pointers are typed by
// the instance precision (float or double); parameters are kept in FP64 (host side
// and FP64 reductions) and in the coefficient blocks of both precisions.
struct DevInst {
    void* W[5];      // state at the start of the step: He, p, Mx, My, C
    void* W1[5];     // stage-1 output (also the R(W) output of the rhs call)
    void* W2[5];     // stage-2 output
    void* phi[2];    // potential minus the applied-field potential, double buffered
    void* S;         // lagged dFs/dt
    void* kf[3];     // written by stage 1 for stages 2 and 3: the Kelvin force (x, y) of the
                     // step (the potential and the step-start state do not change within
                     // it) and the liquid fraction of the step-start state; from stage 3
                     // to the next step's stage 1, kf[0] holds the permeability of the
                     // state (for the magnetic phase)
    double* part;    // [ntile_stage][NPART]
    double* mpart;   // residual partials of the magnetic phase (one per magnetic tile, or one
                     // per stage tile when stage 1 runs the phase), then the convergence flag
    double* result;  // [NRES]
    int32_t nx, ny, pitch;
    int32_t per_x, per_y;
    int32_t tbc[4], mbc[4];
    int32_t ntile_stage, ntile_mag;
    int32_t col_height;  // column of the height observable
    int32_t heat_on;     // south wall is a fixed-temperature wall
    double tval[4];
    double wet[4];   // (4 / xi) cos(contact angle) per wall (0: mirror)
    double rho[3], mu_[3], lam[3], cp[3], chi[3];
    double latent, tm, tl, dx, dt, dts, cpref, qg, tau_g, beta, kappa, mu0, h0x, h0y, xi;   // tm, tl: Ts, Tl
    double grav[2];
    double vc;       // 1 - rho_s / rho_l
    double mag_kdt;  // D dtau / dx^2 (magnetic pseudo-time solve)
    double mag_tol;  // ||r||_2 target of the convergence-controlled magnetic phase
    Coef<float> cf;  // the parameters above in FP32 (FP32 instances)
    Coef<double> cd; // and in FP64 (FP64 instances)
};

template <typename T>
__host__ __device__ inline const Coef<T>& coef(const DevInst& I);
template <>
__host__ __device__ inline const Coef<float>& coef<float>(const DevInst& I) { return I.cf; }
template <>
__host__ __device__ inline const Coef<double>& coef<double>(const DevInst& I) { return I.cd; }

// launchers (lbfs_kernels.hip); all enqueue on `stream`, return hipError_t
// stage kernel of tile shape `shape` (index into the precision's table); stage 0 is
// the plain right-hand side R(W) into W1
// (with e0 / e1 the launch records the kernel's start / end time into them)
template <typename T>
hipError_t launch_stage(int shape, int stage, int pidx, const DevInst* insts, const Tile* tiles, int ntiles,
                        hipStream_t stream, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// stage 1 with the step's magnetic phase fused in front of it (red-black sweeps of
// each stage tile plus a halo of 2*MAG_KMAX+3 in LDS, nsweeps <= MAG_KMAX): reads the
// potential buffer pidx, writes the other one and one residual partial per stage tile
template <typename T>
hipError_t launch_stage_fused(int shape, int pidx, int nsweeps, double omega, const DevInst* insts,
                              const Tile* tiles, int ntiles, hipStream_t stream, hipEvent_t e0 = nullptr,
                              hipEvent_t e1 = nullptr);
// magnetic phase: permeability, nsweeps red-black sweeps with factor omega, and the
// residual partials when residual != 0, on tiles of MAG_SHAPES[shape]. Reads the
// potential buffer *pidx and flips *pidx once per launch. With muin != 0 the
// permeability is read from kf[0], which stage 3 fills with that of the state it
// writes; the caller passes muin only when no other write of the state came since.
// With gate != 0 an instance whose convergence flag is set only copies its potential
// to the other buffer (the flip stays uniform) and keeps its residual partials.
template <typename T>
hipError_t launch_mag(int shape, int nsweeps, double omega, int residual, int muin, int* pidx, const DevInst* insts,
                      const Tile* tiles, int ntiles, hipStream_t stream, hipEvent_t e0 = nullptr,
                      hipEvent_t e1 = nullptr, int gate = 0);
// magnetic phase by the LBFS pseudo-time solve: permeability, nsteps SSP-RK3 steps of
// Eq. 17 (rate factor mag_kdt of each instance) and the residual partials when
// residual != 0, on tiles of MAG_SHAPES[shape]; buffers as launch_mag.
template <typename T>
hipError_t launch_mag_lbfs(int shape, int nsteps, int residual, int* pidx, const DevInst* insts,
                           const Tile* tiles, int ntiles, hipStream_t stream, hipEvent_t e0 = nullptr,
                           hipEvent_t e1 = nullptr, int gate = 0);
// convergence flag of each instance: 1 when the residual of its last magnetic launch
// is at most mag_tol (one workgroup per instance)
hipError_t launch_mag_gate(const DevInst* insts, int ninst, hipStream_t stream);
// geometric multigrid for the compact magnetic system (lbfs_kernels.hip, one instance):
// the coarsest level has at most MG_COARSE x MG_COARSE cells and is solved in the LDS of
// one workgroup
constexpr int MG_COARSE = 32;
template <typename T>
hipError_t launch_mg_setup0(const DevInst* insts, int nx, int ny, T* mu_tmp, T* wx, T* wy, T* f, hipStream_t stream,
                            hipEvent_t e0 = nullptr);
template <typename T>
hipError_t launch_mg_coarsen(int nxf, int nyf, const T* wxf, const T* wyf, int nxc, int nyc, T* wxc, T* wyc,
                             const int* geom, hipStream_t stream);
template <typename T>
hipError_t launch_mg_smooth(int nx, int ny, int pitch, T* u, const T* f, const T* wx, const T* wy, int sweeps,
                            hipStream_t stream);
template <typename T>
hipError_t launch_mg_restrict(int nxf, int nyf, int pitchf, const T* uf, const T* ff, const T* wxf, const T* wyf,
                              int nxc, int nyc, T* fc, T* uc, hipStream_t stream);
// fixed_walls: bit w set where wall w (W, E, S, N) holds the potential (the correction
// vanishes there); other walls are insulating. geom (coarsening and prolongation): the
// fine level's cell width in level-0 cells, the widths of its last column and last row,
// and those of the coarse level's last column and last row.
template <typename T>
hipError_t launch_mg_prolong(int nxf, int nyf, int pitchf, T* uf, int nxc, int nyc, const T* uc, int fixed_walls,
                             const int* geom, hipStream_t stream);
template <typename T>
hipError_t launch_mg_coarsest(int nx, int ny, int pitch, T* u, const T* f, const T* wx, const T* wy, int sweeps,
                              double omega, hipStream_t stream);
// per-tile FP64 partial sums of the observables over stage tiles of shape `shape`
template <typename T>
hipError_t launch_state_partials(int shape, const DevInst* insts, const Tile* tiles, int ntiles, hipStream_t stream);
// mres_stage != 0: the last magnetic residual partials came from stage 1 (one per stage
// tile), else from a magnetic launch (one per magnetic tile)
hipError_t launch_reduce(const DevInst* insts, int ninst, hipStream_t stream, int mres_stage = 0);
template <typename T>
hipError_t launch_init_fields(const DevInst* insts, const Tile* tiles, int ntiles, int kind,
                              double c_init, double t_init, double cx, double cy, double r,
                              hipStream_t stream);
template <typename T>
hipError_t launch_derived(const DevInst* insts, const Tile* tiles, int ntiles, hipStream_t stream);
// local wall heat flux of instance 0 (nx FP64 values into out)
template <typename T>
hipError_t launch_wall_profile(const DevInst* insts, int nx, double* out, hipStream_t stream);

}  // namespace lbfs

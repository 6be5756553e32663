// lbfs_api.hip -- host side of the C ABI declared in include/lbfs.h.
//
// The solver state lives in one caller-owned device buffer, carved into 256-byte
// aligned segments: the instance descriptor, the tile lists, FP64 partials and
// results, and 18 SoA fields (W, W1, W2 of 5 fields each, phi' twice, S) with the row
// pitch padded to 64 elements. No device allocation happens inside the library.
#include "lbfs.h"
#include "lbfs_internal.hpp"

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

using namespace lbfs;

namespace {

constexpr size_t ALIGN = 256;
constexpr int NFIELDS = 18;   // W[5], W1[5], W2[5], phi[0], S, phi[1]
constexpr uint32_t CKPT_MAGIC = 0x5346424cu;   // "LBFS"

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
    int pitch = 0;
    size_t esize = 0, field_bytes = 0;
    int tiles_stage_x = 0, tiles_stage_y = 0, tiles_mag_x = 0, tiles_mag_y = 0, tiles_pt_x = 0, tiles_pt_y = 0;
    int mag_big = 0, mag_tx = 0, mag_ty = 0;
    size_t off_inst = 0, off_tstage = 0, off_tmag = 0, off_tpt = 0, off_part = 0, off_mpart = 0, off_res = 0,
           off_fields = 0, total = 0;
    int ntile_stage() const { return tiles_stage_x * tiles_stage_y; }
    int ntile_mag() const { return tiles_mag_x * tiles_mag_y; }
    int ntile_pt() const { return tiles_pt_x * tiles_pt_y; }
};

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int validate(const lbfs_params* p)
{
    if (!p) return LBFS_E_INVAL;
    if (p->abi_version != LBFS_ABI_VERSION) return LBFS_E_ABI;
    if (p->nx < 4 || p->ny < 4 || p->nx > (1 << 20) || p->ny > (1 << 20)) return LBFS_E_INVAL;
    if (p->precision != LBFS_FP32 && p->precision != LBFS_FP64) return LBFS_E_INVAL;
    if (!finite_pos(p->dx) || !finite_pos(p->dt)) return LBFS_E_INVAL;
    if (p->dt_stream != 0.0 && std::fabs(p->dt_stream - 0.5 * p->dx) > 1e-12 * p->dx) return LBFS_E_INVAL;
    for (int k = 0; k < 3; k++) {
        if (!finite_pos(p->rho[k]) || !finite_pos(p->mu[k]) || !finite_pos(p->cp[k]) ||
            !finite_pos(p->lambda[k]))
            return LBFS_E_INVAL;
        if (!std::isfinite(p->chi[k]) || p->chi[k] <= -1.0) return LBFS_E_INVAL;
    }
    if (!std::isfinite(p->latent) || p->latent < 0.0) return LBFS_E_INVAL;
    if (!std::isfinite(p->t_melt) || !std::isfinite(p->t_init)) return LBFS_E_INVAL;
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
    }
    if (p->sweeps < 0 || p->sweeps > 1000) return LBFS_E_INVAL;
    if (!(p->sor_omega > 0.0 && p->sor_omega < 2.0)) return LBFS_E_INVAL;
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
    if (dmax * p->dt / (p->dx * p->dx) > 0.5) return LBFS_E_INVAL;
    if (std::sqrt(1.0 / 3.0) * p->dt / p->dx > 1.0) return LBFS_E_INVAL;
    return LBFS_OK;
}

Layout make_layout(const lbfs_params* p)
{
    Layout L;
    L.esize = p->precision == LBFS_FP64 ? 8 : 4;
    L.pitch = (int)align_up((size_t)p->nx, 64);
    L.field_bytes = align_up((size_t)L.pitch * p->ny * L.esize, ALIGN);
    const int stx = p->precision == LBFS_FP64 ? STAGE_TX_F64 : STAGE_TX_F32;
    const int sty = p->precision == LBFS_FP64 ? STAGE_TY_F64 : STAGE_TY_F32;
    L.tiles_stage_x = (p->nx + stx - 1) / stx;
    L.tiles_stage_y = (p->ny + sty - 1) / sty;
    L.mag_big = (size_t)p->nx * p->ny > (size_t)512 * 512 ? 1 : 0;
    L.mag_tx = L.mag_big ? MAG_BIG_TX : MAG_SMALL_TX;
    L.mag_ty = L.mag_big ? MAG_BIG_TY : MAG_SMALL_TY;
    L.tiles_mag_x = (p->nx + L.mag_tx - 1) / L.mag_tx;
    L.tiles_mag_y = (p->ny + L.mag_ty - 1) / L.mag_ty;
    L.tiles_pt_x = (p->nx + PT_TX - 1) / PT_TX;
    L.tiles_pt_y = (p->ny + PT_TY - 1) / PT_TY;
    size_t off = 0;
    L.off_inst = off; off = align_up(off + sizeof(DevInst), ALIGN);
    L.off_tstage = off; off = align_up(off + sizeof(Tile) * L.ntile_stage(), ALIGN);
    L.off_tmag = off; off = align_up(off + sizeof(Tile) * L.ntile_mag(), ALIGN);
    L.off_tpt = off; off = align_up(off + sizeof(Tile) * L.ntile_pt(), ALIGN);
    L.off_part = off; off = align_up(off + sizeof(double) * NPART * L.ntile_stage(), ALIGN);
    L.off_mpart = off; off = align_up(off + sizeof(double) * L.ntile_mag(), ALIGN);
    L.off_res = off; off = align_up(off + sizeof(double) * NRES, ALIGN);
    L.off_fields = off; off += L.field_bytes * NFIELDS;
    L.total = off + ALIGN;   // room to align the caller's base pointer
    return L;
}

}  // namespace

struct lbfs_solver {
    lbfs_params p;
    Layout L;
    hipStream_t stream = nullptr;
    char* base = nullptr;
    DevInst hinst{};
    DevInst* dinst = nullptr;
    Tile* dtiles_stage = nullptr;
    Tile* dtiles_mag = nullptr;
    Tile* dtiles_pt = nullptr;
    hipGraph_t graph[2] = {nullptr, nullptr};          // one captured step per potential buffer
    hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
    bool use_graph = true;
    int phase = 0;                       // potential buffer holding the current phi'
    int phi_field() const { return phase ? 17 : 15; }
    double* hres = nullptr;      // pinned copy of the results
    void* staging = nullptr;     // pinned field staging (nx*ny elements of 8 bytes)
    double t = 0.0;
    int64_t step = 0;
    double vol0 = 0.0;
    bool stepped_since_observe = false;
    void* field(int k) const { return base + L.off_fields + L.field_bytes * (size_t)k; }
    bool f64() const { return p.precision == LBFS_FP64; }
};

#define HIPCHK(x)                                   \
    do {                                            \
        if ((x) != hipSuccess) return LBFS_E_DEVICE; \
    } while (0)

namespace {

hipError_t launch_mag_phase(lbfs_solver* s, int nsweeps, double omega, int residual)
{
    const int nm = s->L.ntile_mag();
    return s->f64()
        ? launch_mag<double>(s->L.mag_big, nsweeps, omega, residual, &s->phase, s->dinst, s->dtiles_mag, nm, s->stream)
        : launch_mag<float>(s->L.mag_big, nsweeps, omega, residual, &s->phase, s->dinst, s->dtiles_mag, nm, s->stream);
}

hipError_t launch_stage_k(lbfs_solver* s, int stage)
{
    const int ns = s->L.ntile_stage();
    return s->f64() ? launch_stage<double>(stage, s->phase, s->dinst, s->dtiles_stage, ns, s->stream)
                    : launch_stage<float>(stage, s->phase, s->dinst, s->dtiles_stage, ns, s->stream);
}

hipError_t launch_state_part(lbfs_solver* s)
{
    const int ns = s->L.ntile_stage();
    return s->f64() ? launch_state_partials<double>(s->dinst, s->dtiles_stage, ns, s->stream)
                    : launch_state_partials<float>(s->dinst, s->dtiles_stage, ns, s->stream);
}

// one time step: magnetic phase and three Runge-Kutta stages (the observables of the
// state are summed when they are read)
hipError_t enqueue_step(lbfs_solver* s)
{
    hipError_t e = launch_mag_phase(s, s->p.sweeps, s->p.sor_omega, 1);
    for (int st = 1; st <= 3 && e == hipSuccess; st++) e = launch_stage_k(s, st);
    return e;
}

// residual of the magnetic system of the current state, synchronously
int mag_residual_now(lbfs_solver* s, double* out)
{
    HIPCHK(launch_mag_phase(s, 0, 1.0, 1));
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
    const size_t es = s->L.esize, nx = s->p.nx, ny = s->p.ny;
    HIPCHK(hipMemcpy2DAsync(s->staging, nx * es, s->field(k), (size_t)s->L.pitch * es, nx * es, ny,
                            hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    for (size_t q = 0; q < nx * ny; q++)
        host[q] = s->f64() ? static_cast<double*>(s->staging)[q] : (double)static_cast<float*>(s->staging)[q];
    return LBFS_OK;
}

int copy_field_in(lbfs_solver* s, int k, const double* host)
{
    const size_t es = s->L.esize, nx = s->p.nx, ny = s->p.ny;
    for (size_t q = 0; q < nx * ny; q++) {
        if (s->f64()) static_cast<double*>(s->staging)[q] = host[q];
        else static_cast<float*>(s->staging)[q] = (float)host[q];
    }
    HIPCHK(hipMemcpy2DAsync(s->field(k), (size_t)s->L.pitch * es, s->staging, nx * es, nx * es, ny,
                            hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
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
    for (int w = 0; w < 4; w++) p->mag_bc[w] = LBFS_MBC_FIXED;
    p->sweeps = 4;
    p->sor_omega = 1.0;
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

int lbfs_init(const lbfs_params* p, void* dev_buf, size_t bytes, void* stream, lbfs_solver** out)
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
    if (s->p.dt_stream == 0.0) s->p.dt_stream = 0.5 * p->dx;
    if (s->p.init_check == 0) s->p.init_check = 50;
    s->L = L;
    s->stream = static_cast<hipStream_t>(stream);
    s->base = reinterpret_cast<char*>(align_up(reinterpret_cast<uintptr_t>(dev_buf), ALIGN));
    s->dinst = reinterpret_cast<DevInst*>(s->base + L.off_inst);
    s->dtiles_stage = reinterpret_cast<Tile*>(s->base + L.off_tstage);
    s->dtiles_mag = reinterpret_cast<Tile*>(s->base + L.off_tmag);
    s->dtiles_pt = reinterpret_cast<Tile*>(s->base + L.off_tpt);
    auto fail = [&](int code) {
        lbfs_destroy(s);
        return code;
    };
    if (hipHostMalloc(&s->hres, sizeof(double) * NRES, hipHostMallocDefault) != hipSuccess) return fail(LBFS_E_DEVICE);
    if (hipHostMalloc(&s->staging, (size_t)p->nx * p->ny * 8, hipHostMallocDefault) != hipSuccess)
        return fail(LBFS_E_DEVICE);

    // descriptor
    DevInst& I = s->hinst;
    std::memset(&I, 0, sizeof I);
    for (int k = 0; k < 5; k++) {
        I.W[k] = s->field(k);
        I.W1[k] = s->field(5 + k);
        I.W2[k] = s->field(10 + k);
    }
    I.phi[0] = s->field(15);
    I.phi[1] = s->field(17);
    I.S = s->field(16);
    I.part = reinterpret_cast<double*>(s->base + L.off_part);
    I.mpart = reinterpret_cast<double*>(s->base + L.off_mpart);
    I.result = reinterpret_cast<double*>(s->base + L.off_res);
    I.nx = p->nx;
    I.ny = p->ny;
    I.pitch = L.pitch;
    I.per_x = p->periodic[0];
    I.per_y = p->periodic[1];
    for (int w = 0; w < 4; w++) {
        I.tbc[w] = p->thermal_bc[w];
        I.mbc[w] = p->mag_bc[w];
        I.tval[w] = p->thermal_val[w];
    }
    I.ntile_stage = L.ntile_stage();
    I.ntile_mag = L.ntile_mag();
    int col = (int)std::floor(p->drop_cx / p->dx);
    I.col_height = col < 0 ? 0 : (col > p->nx - 1 ? p->nx - 1 : col);
    I.heat_on = (!p->periodic[1] && p->thermal_bc[2] == LBFS_TBC_FIXED) ? 1 : 0;
    for (int k = 0; k < 3; k++) {
        I.rho[k] = p->rho[k]; I.mu_[k] = p->mu[k]; I.lam[k] = p->lambda[k]; I.cp[k] = p->cp[k]; I.chi[k] = p->chi[k];
    }
    I.latent = p->latent;
    I.tm = p->t_melt;
    I.dx = p->dx;
    I.dt = p->dt;
    I.dts = s->p.dt_stream;
    I.cpref = 0.5 * (p->cp[0] + p->cp[1]);
    I.qg = p->mobility / ((p->tau_g - 0.5) * s->p.dt_stream);   // M_c = (tau_g - 1/2) Q_g delta_t
    I.tau_g = p->tau_g;
    I.beta = 12.0 * p->sigma / p->xi;
    I.kappa = 1.5 * p->xi * p->sigma;
    I.mu0 = p->mu0;
    const double th = p->field_angle_deg * M_PI / 180.0;
    I.h0x = p->h0 * std::cos(th);
    I.h0y = p->h0 * std::sin(th);
    I.xi = p->xi;
    I.grav[0] = p->gravity[0];
    I.grav[1] = p->gravity[1];
    I.vc = 1.0 - p->rho[0] / p->rho[1];

    std::vector<Tile> ts, tm, tp;
    {
        const int stx = s->f64() ? STAGE_TX_F64 : STAGE_TX_F32, sty = s->f64() ? STAGE_TY_F64 : STAGE_TY_F32;
        for (int ty = 0; ty < L.tiles_stage_y; ty++)
            for (int tx = 0; tx < L.tiles_stage_x; tx++)
                ts.push_back(Tile{0, tx * stx, ty * sty, (int)ts.size()});
        for (int ty = 0; ty < L.tiles_mag_y; ty++)
            for (int tx = 0; tx < L.tiles_mag_x; tx++)
                tm.push_back(Tile{0, tx * L.mag_tx, ty * L.mag_ty, (int)tm.size()});
        for (int ty = 0; ty < L.tiles_pt_y; ty++)
            for (int tx = 0; tx < L.tiles_pt_x; tx++)
                tp.push_back(Tile{0, tx * PT_TX, ty * PT_TY, (int)tp.size()});
    }
    if (hipMemcpyAsync(s->dinst, &I, sizeof I, hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(s->dtiles_stage, ts.data(), sizeof(Tile) * ts.size(), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(s->dtiles_mag, tm.data(), sizeof(Tile) * tm.size(), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(s->dtiles_pt, tp.data(), sizeof(Tile) * tp.size(), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemsetAsync(s->base + L.off_part, 0, L.off_fields - L.off_part, s->stream) != hipSuccess ||
        hipMemsetAsync(s->base + L.off_fields, 0, L.field_bytes * NFIELDS, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return fail(LBFS_E_DEVICE);

    hipError_t e = s->f64()
        ? launch_init_fields<double>(s->dinst, s->dtiles_pt, L.ntile_pt(), p->init_kind, p->c_init, p->t_init,
                                     p->drop_cx, p->drop_cy, p->drop_radius, s->stream)
        : launch_init_fields<float>(s->dinst, s->dtiles_pt, L.ntile_pt(), p->init_kind, p->c_init, p->t_init,
                                    p->drop_cx, p->drop_cy, p->drop_radius, s->stream);
    if (e != hipSuccess) return fail(LBFS_E_DEVICE);

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
        if (launch_mag_phase(s, k, om, 0) != hipSuccess) return fail(LBFS_E_DEVICE);
        used += k;
        const double r_prev = r;
        if (mag_residual_now(s, &r) != LBFS_OK) return fail(LBFS_E_DEVICE);
        if (!std::isfinite(r)) return fail(LBFS_E_NONFINITE);
        if (r > 0.98 * r_prev) break;   // stagnated at the round-off floor of the precision
    }
    // observables of the initial state (also the reference volume A0)
    if (launch_state_part(s) != hipSuccess || launch_reduce(s->dinst, 1, s->stream) != hipSuccess ||
        hipMemcpyAsync(s->hres, I.result, sizeof(double) * NRES, hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return fail(LBFS_E_DEVICE);
    s->vol0 = s->hres[RES_CT] * p->dx * p->dx;
    s->hres[RES_MAGR2] = r * r;
    const char* ng = std::getenv("LBFS_NO_GRAPH");
    s->use_graph = s->stream != nullptr && !(ng && ng[0] == '1');
    *out = s;
    return LBFS_OK;
}

// capture one time step starting from potential buffer `ph` into a HIP graph (once
// per buffer); replays cost one launch per step
static int ensure_graph(lbfs_solver* s, int ph)
{
    if (!s->use_graph || s->graph_exec[ph]) return LBFS_OK;
    const int saved = s->phase;
    s->phase = ph;
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(s->stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
        s->phase = saved;
        return LBFS_E_DEVICE;
    }
    const hipError_t e = enqueue_step(s);
    const hipError_t ec = hipStreamEndCapture(s->stream, &g);
    s->phase = saved;
    if (e != hipSuccess || ec != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return LBFS_E_DEVICE;
    }
    if (hipGraphInstantiate(&s->graph_exec[ph], g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        s->graph_exec[ph] = nullptr;
        return LBFS_E_DEVICE;
    }
    s->graph[ph] = g;
    return LBFS_OK;
}

// potential-buffer flips of one step (one per magnetic launch)
static int step_flips(const lbfs_solver* s)
{
    const int launches = s->p.sweeps == 0 ? 1 : (s->p.sweeps + MAG_KMAX - 1) / MAG_KMAX;
    return launches & 1;
}

// one step, as a graph replay when graphs are on
static hipError_t run_step(lbfs_solver* s)
{
    if (s->use_graph) {
        const int ph = s->phase;
        if (ensure_graph(s, ph) != LBFS_OK) return hipErrorUnknown;
        const hipError_t e = hipGraphLaunch(s->graph_exec[ph], s->stream);
        s->phase = ph ^ step_flips(s);
        return e;
    }
    return enqueue_step(s);
}

int lbfs_step(lbfs_solver* s, int32_t nsteps)
{
    if (!s) return LBFS_E_STATE;
    if (nsteps < 0) return LBFS_E_INVAL;
    for (int n = 0; n < nsteps; n++) {
        if (run_step(s) != hipSuccess) return LBFS_E_DEVICE;
        s->t += s->p.dt;
        s->step += 1;
        s->stepped_since_observe = true;
    }
    return LBFS_OK;
}

int lbfs_step_profiled(lbfs_solver* s, int32_t nsteps, int32_t sample_every, double* kernel_ms,
                       int32_t* launches)
{
    if (!s) return LBFS_E_STATE;
    if (nsteps < 0 || sample_every < 1 || !kernel_ms || !launches) return LBFS_E_INVAL;
    const int nsample = (nsteps + sample_every - 1) / sample_every;
    if (nsample > 4096) return LBFS_E_INVAL;

    const int per_step = 4;
    std::vector<hipEvent_t> ev((size_t)nsample * per_step * 2, nullptr);
    std::vector<int> kind((size_t)nsample * per_step, 0);
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto& f : ev)
                if (f) (void)hipEventDestroy(f);
            return LBFS_E_DEVICE;
        }
    int rc = LBFS_OK;
    size_t slot = 0;
    auto timed = [&](int k, bool on, auto&& launch) -> hipError_t {
        if (on) {
            kind[slot] = k;
            hipError_t e = hipEventRecord(ev[2 * slot], s->stream);
            if (e != hipSuccess) return e;
        }
        hipError_t e = launch();
        if (e != hipSuccess) return e;
        if (on) {
            e = hipEventRecord(ev[2 * slot + 1], s->stream);
            slot++;
        }
        return e;
    };
    for (int n = 0; n < nsteps && rc == LBFS_OK; n++) {
        const bool on = n % sample_every == 0;
        hipError_t e;
        if (on) {
            e = timed(LBFS_K_MAG, on, [&] { return launch_mag_phase(s, s->p.sweeps, s->p.sor_omega, 1); });
            for (int st = 1; st <= 3 && e == hipSuccess; st++)
                e = timed(LBFS_K_STAGE1 + st - 1, on, [&] { return launch_stage_k(s, st); });
        } else {
            e = run_step(s);
        }
        if (e != hipSuccess) rc = LBFS_E_DEVICE;
        s->t += s->p.dt;
        s->step += 1;
        s->stepped_since_observe = true;
    }
    if (rc == LBFS_OK && hipStreamSynchronize(s->stream) != hipSuccess) rc = LBFS_E_DEVICE;
    for (int k = 0; k < LBFS_NKERNELS; k++) {
        kernel_ms[k] = 0.0;
        launches[k] = 0;
    }
    if (rc == LBFS_OK)
        for (size_t q = 0; q < slot; q++) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, ev[2 * q], ev[2 * q + 1]) != hipSuccess) {
                rc = LBFS_E_DEVICE;
                break;
            }
            kernel_ms[kind[q]] += ms;
            launches[kind[q]] += 1;
        }
    for (int k = 0; k < LBFS_NKERNELS; k++)
        if (launches[k] > 0) kernel_ms[k] /= launches[k];
    for (auto& e : ev) (void)hipEventDestroy(e);
    return rc;
}

int lbfs_observe(lbfs_solver* s, lbfs_observables* o)
{
    if (!s || !o) return s ? LBFS_E_INVAL : LBFS_E_STATE;
    if (s->stepped_since_observe) {
        HIPCHK(launch_state_part(s));
        HIPCHK(launch_reduce(s->dinst, 1, s->stream));
        HIPCHK(hipMemcpyAsync(s->hres, s->hinst.result, sizeof(double) * NRES, hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        s->stepped_since_observe = false;
    }
    const double* r = s->hres;
    const double dA = s->p.dx * s->p.dx;
    std::memset(o, 0, sizeof *o);
    o->t = s->t;
    o->step = s->step;
    o->volume = r[RES_CT] * dA;
    o->volume0 = s->vol0;
    o->liquid_fraction = r[RES_CT] > 0.0 ? r[RES_CTFL] / r[RES_CT] : 0.0;
    o->solid_ratio = s->vol0 > 0.0 ? r[RES_FS] * dA / s->vol0 : 0.0;
    o->mag_residual = std::sqrt(r[RES_MAGR2]);
    o->umax = r[RES_UMAX];
    o->umax_drop = r[RES_UDROP];
    o->height = r[RES_HEIGHT] * s->p.dx;
    o->wall_heat = r[RES_HEAT];
    o->nonfinite = r[RES_NONFINITE] != 0.0 || !std::isfinite(r[RES_CT]) ? 1 : 0;
    return o->nonfinite ? LBFS_E_NONFINITE : LBFS_OK;
}

int lbfs_rhs(lbfs_solver* s, double* host_R)
{
    if (!s) return LBFS_E_STATE;
    if (!host_R) return LBFS_E_INVAL;
    HIPCHK(launch_stage_k(s, 0));
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
    if (nsweeps < 0 || !(omega > 0.0 && omega < 2.0)) return LBFS_E_INVAL;
    HIPCHK(launch_mag_phase(s, nsweeps, omega, 0));
    double r = 0.0;
    const int rc = mag_residual_now(s, &r);
    if (rc != LBFS_OK) return rc;
    if (residual) *residual = r;
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
}  // namespace

size_t lbfs_checkpoint_bytes(const lbfs_solver* s)
{
    if (!s) return 0;
    return sizeof(CkptHeader) + 7 * (size_t)s->p.nx * s->p.ny * s->L.esize;
}

int lbfs_save_state(lbfs_solver* s, void* host, size_t bytes)
{
    if (!s) return LBFS_E_STATE;
    if (!host || bytes < lbfs_checkpoint_bytes(s)) return LBFS_E_INVAL;
    CkptHeader h{CKPT_MAGIC, LBFS_ABI_VERSION, s->p.nx, s->p.ny, s->p.precision, 0, s->t, s->vol0, s->step};
    std::memcpy(host, &h, sizeof h);
    char* dst = static_cast<char*>(host) + sizeof h;
    const size_t es = s->L.esize, row = (size_t)s->p.nx * es, fb = row * s->p.ny;
    for (int q = 0; q < 7; q++) {
        const int f = CKPT_FIELDS[q] == -2 ? s->phi_field() : CKPT_FIELDS[q];
        HIPCHK(hipMemcpy2DAsync(s->staging, row, s->field(f), (size_t)s->L.pitch * es, row, s->p.ny,
                                hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        std::memcpy(dst + q * fb, s->staging, fb);
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
    const size_t es = s->L.esize, row = (size_t)s->p.nx * es, fb = row * s->p.ny;
    for (int q = 0; q < 7; q++) {
        std::memcpy(s->staging, src + q * fb, fb);
        const int f = CKPT_FIELDS[q] == -2 ? s->phi_field() : CKPT_FIELDS[q];
        HIPCHK(hipMemcpy2DAsync(s->field(f), (size_t)s->L.pitch * es, s->staging, row, row, s->p.ny,
                                hipMemcpyHostToDevice, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    s->t = h.t;
    s->step = h.step;
    s->vol0 = h.vol0;
    return LBFS_OK;
}

void lbfs_destroy(lbfs_solver* s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    for (int k = 0; k < 2; k++) {
        if (s->graph_exec[k]) (void)hipGraphExecDestroy(s->graph_exec[k]);
        if (s->graph[k]) (void)hipGraphDestroy(s->graph[k]);
    }
    if (s->hres) (void)hipHostFree(s->hres);
    if (s->staging) (void)hipHostFree(s->staging);
    delete s;
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

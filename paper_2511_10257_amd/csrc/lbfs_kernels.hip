// lbfs_kernels.hip -- gfx950 kernels of the enthalpy LBFS time step.
//
// Kernels (all driven by tile lists, see lbfs_internal.hpp):
//   k_stage<T,TX,TY,NT,ST>  fused Runge-Kutta stage: LDS-staged halo of the cell
//                           fields, Eq. 8 / Eq. 11 derived fields, chemical potential,
//                           central gradients, Kelvin force (stage 1; stages 2 and 3
//                           read it), LBFS fluxes of every face of the tile, sources
//                           (Eq. 41), residual (Eq. 42) and the SSP-RK3 combination
//                           (Eq. 46); the last stage also applies Eq. 8 for the lagged
//                           dFs/dt and leaves the new state's permeability for the
//                           next step's sweeps.
//   k_state_partials        FP64 per-tile partial sums of the observables of a state.
//   k_mag_fused             permeability (Eq. 2 with Eq. 11, or read where stage 3
//                           left it), red-black sweeps of the compact magnetic system
//                           (temporally blocked in LDS) and the FP64 residual.
//   k_mag_lbfs              the same phase by the magnetic LBFS pseudo-time solve
//                           (Eq. 17, SSP-RK3 steps temporally blocked in LDS).
//   k_reduce                fixed-order FP64 reduction of the partials per instance.
//   k_mg_*                  geometric multigrid for the compact magnetic system.
//   k_init_fields, k_derived, k_wall_profile (local wall heat flux, Sec. 5.2)
//
// The path is a stencil: a few hundred flops per face over ~70 bytes per cell and
// stage, no dense contraction, so no MFMA. Fields are SoA with a padded row pitch;
// the stage kernel reads each tile plus a 3-cell halo once into LDS.
#include "lbfs_face.hpp"
#include "lbfs_internal.hpp"

#include <hip/hip_ext.h>
#include <ratio>
#include <type_traits>

namespace lbfs {

// Launch on `stream`; with timing events the launch timestamps the kernel's own start
// and end into them (hipExtLaunchKernelGGL), so the measured duration holds no
// dispatch gap.
template <typename K, typename... A>
hipError_t launch_timed(K kernel, dim3 grid, dim3 block, hipStream_t stream, hipEvent_t e0, hipEvent_t e1,
                        A... args)
{
    if (e0 || e1)
        hipExtLaunchKernelGGL(kernel, grid, block, 0, stream, e0, e1, 0, args...);
    else
        hipLaunchKernelGGL(kernel, grid, block, 0, stream, args...);
    return hipGetLastError();
}

// ------------------------------------------------------------------ helpers

// Field pointers live in the instance descriptor as generic pointers; cast them to the
// global address space so that accesses compile to global (not flat) memory ops.
#define GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ GLOBAL T* gp(void* p) { return (GLOBAL T*)p; }

// Eq. 11: property of the solid / liquid / gas mixture
template <typename T>
__device__ __forceinline__ T mix3(const T* g, T fs, T ct)
{
    return fs * g[0] + (T(1) - fs) * ct * g[1] + (T(1) - fs) * (T(1) - ct) * g[2];
}

// Eq. 2 with Eq. 11: the permeability mu0 (1 + chi) of a cell from its clamped order
// parameter and liquid fraction (the magnetic kernels, and stage 3 for the next step)
template <typename T>
__device__ __forceinline__ T mag_permeability(const Coef<T>& K, T ct, T Fl)
{
    return K.mu0 * (T(1) + mix3<T>(K.chi, ct * (T(1) - Fl), ct));
}

template <typename T>
struct Prim {
    T p, u, v, rho, C, Tt, He, mu, lam, cp, fs, Fl;
};

template <typename T>
__device__ __forceinline__ Prim<T> primitives(const Coef<T>& K, T He, T p, T Mx, T My, T C)
{
    Prim<T> q;
    T Fl;
    enthalpy_state<T>(K, He, C, q.Tt, Fl);
    const T ct = clamp01(C);
    q.Fl = Fl;
    q.fs = ct * (T(1) - Fl);
    q.rho = mix3<T>(K.rho, q.fs, ct);
    q.mu = mix3<T>(K.mu, q.fs, ct);
    q.lam = mix3<T>(K.lam, q.fs, ct);
    q.cp = mix3<T>(K.cp, q.fs, ct);
    const T inv = T(3) * rcp_bounded(q.rho);   // 1 / (rho cs^2)
    q.u = Mx * inv;
    q.v = My * inv;
    q.p = p;
    q.C = C;
    q.He = He;
    return q;
}

// Source cell of grid coordinate g along an axis of n cells: itself, the periodic
// image, or the mirror cell across the wall (then `wall` names it). Coordinates
// further than the 3-cell halo from the domain (only in tiles of tiny domains) are
// clamped: their values never reach an output.
__device__ __forceinline__ int map_axis(int g, int n, int periodic, int wlo, int whi, int& wall)
{
    int s = g;
    wall = -1;
    if (g < 0) {
        if (periodic) s = g + n;
        else { s = -1 - g; wall = wlo; }
    } else if (g >= n) {
        if (periodic) s = g - n;
        else { s = 2 * n - 1 - g; wall = whi; }
    }
    return s < 0 ? 0 : (s >= n ? n - 1 : s);
}

// ------------------------------------------------------------- face flux

// ------------------------------------------------------------- tile order

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2). Map
// dispatch index -> tile so that every XCD works through one contiguous range of the
// (row-major) tile list: neighbouring tiles, whose halos overlap, then share an L2.
__device__ __forceinline__ int xcd_tile(int bid, int n)
{
    constexpr int NXCD = 8;
    const int q = n / NXCD, r = n % NXCD;
    const int x = bid % NXCD, k = bid / NXCD;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// ------------------------------------------------------------- magnetics

// Region of a temporally blocked red-black block: an MTX x MTY tile plus a halo of H
// cells, the potential split by colour (cell (lx, ly) of colour c at
// ph[c][ly * RXH + lx / 2]).
template <int MTX, int MTY, int H_>
struct MagGeom {
    static constexpr int H = H_;
    static constexpr int RX = MTX + 2 * H, RY = MTY + 2 * H, NR = RX * RY;
    static constexpr int RXH = RX / 2, HALF = NR / 2;
    static_assert(RX % 2 == 0, "region rows hold whole red-black pairs");
};

// Permeability (Eq. 2 with Eq. 11) of the tile at (x0, y0) plus a halo of H cells, then
// nsweeps red-black sweeps of the compact magnetic system done in LDS (temporal
// blocking: the region where the sweeps are exact shrinks by one cell per colour pass,
// so cells at least 2 nsweeps from the region edge are exact), and optionally the FP64
// residual of the tile's cells (returned as this thread's share). The final potential
// stays in ph. Each cell update is the same arithmetic as an untiled red-black pass, so
// the result does not depend on the tiling or on which kernel runs the block.
//
// Update of cell c: phi'_c <- (1-w) phi'_c + w sum_f a_f (phi'_nb + phi0_nb - phi0_c) / sum_f a_f,
// a_f = mean(mu) on interior faces, 2 mu_c towards a fixed-potential wall half a cell
// away (where phi' = 0), no term at an insulating wall; phi0 = -(h0x x + h0y y).
//
// Each thread owns fixed cells of both colours and keeps their face weights, constant
// term and 1 / sum of weights in registers; a pass costs four LDS reads and one write
// per cell, and reads only the other colour's array (contiguous, conflict free).
//
// MUIN = 1: the permeability of the state is read from I.kf[0], where stage 3 of the
// step before left it (the same arithmetic on the same values), instead of being
// computed from He and C.
template <typename T, int MTX, int MTY, int NT, int H, int MUIN = 0>
__device__ __forceinline__ double mag_block(const DevInst& I, int x0, int y0, int pin, int nsweeps, double omega,
                                            int residual, T (*ph)[MagGeom<MTX, MTY, H>::HALF], T* mu)
{
    using G = MagGeom<MTX, MTY, H>;
    constexpr int NIT = (G::NR + NT - 1) / NT;       // region cells per thread (load)
    constexpr int NOWN = (G::HALF + NT - 1) / NT;    // owned cells per thread and colour
    const Coef<T>& K = coef<T>(I);
    const int tid = threadIdx.x;
    const int nx = I.nx, ny = I.ny;
    const int ox = x0 - G::H, oy = y0 - G::H;
    const int par0 = (ox + oy) & 1;                  // colour of region cell (0, 0)
    const GLOBAL T* phin = gp<T>(I.phi[pin]);
    const GLOBAL T* He_ = gp<T>(I.W[0]);
    const GLOBAL double* C_ = gp<double>(I.W[4]);
    const GLOBAL T* Mu_ = gp<T>(I.kf[0]);
    // 1. load the region (all loads of this thread in flight together): permeability in
    //    natural layout (0 outside the domain), potential by colour
    {
        T vHe[NIT], vC[NIT], vph[NIT];
        bool vin[NIT];
#pragma unroll
        for (int it = 0; it < NIT; it++) {
            const int r = tid + it * NT;
            const int gx = ox + r % G::RX, gy = oy + r / G::RX;
            int sx = gx, sy = gy;
            bool in = r < G::NR;
            // a periodic axis may be shorter than the halo: wrap as often as needed
            if (gx < 0 || gx >= nx) {
                if (I.per_x) sx = ((gx % nx) + nx) % nx;
                else in = false;
            }
            if (gy < 0 || gy >= ny) {
                if (I.per_y) sy = ((gy % ny) + ny) % ny;
                else in = false;
            }
            in = in && sx >= 0 && sx < nx && sy >= 0 && sy < ny;
            vin[it] = in;
            const size_t o = in ? (size_t)sy * I.pitch + sx : 0;
            if constexpr (MUIN) {
                vHe[it] = Mu_[o];   // (the permeability)
                vC[it] = T(0);
            } else {
                vHe[it] = He_[o];
                vC[it] = T(C_[o]);
            }
            vph[it] = phin[o];
        }
#pragma unroll
        for (int it = 0; it < NIT; it++) {
            const int r = tid + it * NT;
            if (r >= G::NR) break;
            const int lx = r % G::RX, ly = r / G::RX;
            T m = T(0);
            if (vin[it]) {
                if constexpr (MUIN) {
                    m = vHe[it];
                } else {
                    T Tt, Fl;
                    enthalpy_state<T>(K, vHe[it], vC[it], Tt, Fl);
                    m = mag_permeability<T>(K, clamp01(vC[it]), Fl);
                }
            }
            mu[r] = m;
            ph[(par0 + lx + ly) & 1][ly * G::RXH + (lx >> 1)] = vin[it] ? vph[it] : T(0);
        }
    }
    __syncthreads();
    // 2. owned cells: item q = c * NOWN + j is the (tid + j * NT)-th cell of colour c.
    //    Face weights (mean permeability of two domain cells; a fixed-potential wall half
    //    a cell away has weight 2 mu_c, an insulating wall none), the constant part of the
    //    numerator and 1 / sum of the weights; rd = 0 marks a cell that is not updated
    //    (region ring 0 or outside the domain).
    const T hx = K.h0x * K.dx, hy = K.h0y * K.dx;
    T wq[2 * NOWN][4], bq[2 * NOWN], rq[2 * NOWN], pq[2 * NOWN];
    int iq[2 * NOWN], sq[2 * NOWN];   // own index in ph[c], row start of the other colour + shift
#pragma unroll
    for (int q = 0; q < 2 * NOWN; q++) {
        const int c = q / NOWN, k = tid + (q % NOWN) * NT;
        rq[q] = T(0);
        bq[q] = T(0);
        pq[q] = T(0);
        iq[q] = 0;
        sq[q] = 0;
#pragma unroll
        for (int d = 0; d < 4; d++) wq[q][d] = T(0);
        if (k >= G::HALF) continue;
        const int ly = k / G::RXH, kx = k % G::RXH;
        const int sh = (par0 + ly + c) & 1;           // lx = 2 kx + sh
        const int lx = 2 * kx + sh;
        iq[q] = k;
        sq[q] = ly * G::RXH + kx + sh;                 // east neighbour; west is one less
        pq[q] = ph[c][k];
        if (lx < 1 || lx >= G::RX - 1 || ly < 1 || ly >= G::RY - 1) continue;
        const int r = ly * G::RX + lx;
        const T muc = mu[r];
        if (!(muc > T(0))) continue;
        const T mnb[4] = {mu[r - 1], mu[r + 1], mu[r - G::RX], mu[r + G::RX]};   // W, E, S, N
        const T D0[4] = {hx, -hx, hy, -hy};   // phi0_nb - phi0_c across each face
        T bsum = T(0), den = T(0);
#pragma unroll
        for (int d = 0; d < 4; d++) {
            const bool nb_in = mnb[d] > T(0);
            // (same operand order as the mean over the face from its west / south cell)
            const T w = nb_in ? (d == 0 || d == 2 ? T(0.5) * (mnb[d] + muc) : T(0.5) * (muc + mnb[d])) : T(0);
            wq[q][d] = w;
            if (w > T(0)) {
                bsum += w * D0[d];
                den += w;
            } else if (!nb_in && I.mbc[d]) {   // a wall face
                const T ww = T(2) * muc;
                bsum += ww * (T(0.5) * D0[d]);
                den += ww;
            }
        }
        bq[q] = bsum;
        rq[q] = den > T(0) ? T(1) / den : T(0);
    }
    // 3. red-black sweeps: a colour pass reads the other colour's array and writes its
    //    own (the colour is a compile-time constant, so the owned-cell registers are
    //    never indexed dynamically)
    const T om = T(omega);
    auto colour_pass = [&](auto colour) {
        constexpr int c = decltype(colour)::value;
        const T* po = ph[c ^ 1];
#pragma unroll
        for (int j = 0; j < NOWN; j++) {
            constexpr int q0 = c * NOWN;
            const int q = q0 + j;
            if (rq[q] == T(0)) continue;
            const int e = sq[q], k = iq[q];
            const T num = bq[q] + wq[q][0] * po[e - 1] + wq[q][1] * po[e] + wq[q][2] * po[k - G::RXH] +
                          wq[q][3] * po[k + G::RXH];
            pq[q] = (T(1) - om) * pq[q] + om * num * rq[q];
            ph[c][k] = pq[q];
        }
        __syncthreads();
    };
    for (int sw = 0; sw < nsweeps; sw++) {
        colour_pass(std::integral_constant<int, 0>{});
        colour_pass(std::integral_constant<int, 1>{});
    }
    // 4. FP64 residual r_c = sum_f a_f (phi_nb - phi_c) over the owned cells of the tile
    double r2 = 0.0;
    if (residual) {
#pragma unroll
        for (int q = 0; q < 2 * NOWN; q++) {
            if (rq[q] == T(0)) continue;
            const int c = q / NOWN, k = iq[q];
            const int ly = k / G::RXH, lx = 2 * (k % G::RXH) + ((par0 + ly + c) & 1);
            const int tx = lx - G::H, ty = ly - G::H;
            if (tx < 0 || tx >= MTX || ty < 0 || ty >= MTY || x0 + tx >= nx || y0 + ty >= ny) continue;
            const T* po = ph[c ^ 1];
            const int e = sq[q];
            const double res = double(bq[q]) + double(wq[q][0]) * double(po[e - 1]) +
                               double(wq[q][1]) * double(po[e]) + double(wq[q][2]) * double(po[k - G::RXH]) +
                               double(wq[q][3]) * double(po[k + G::RXH]) - double(pq[q]) / double(rq[q]);
            r2 += res * res;
        }
    }
    return r2;
}

// ------------------------------------------------------------- stage kernel

// cell fields of the region in LDS: the first Q_P are read until the end of the stage;
// p, mu, lambda, phi' and mu_c (after them) are dead once the face fluxes are computed,
// and the fluxes take their place
enum { Q_U = 0, Q_V, Q_RHO, Q_C, Q_T, Q_HE, Q_CP, Q_P, Q_MU, Q_LAM, Q_PHI, NQ };

template <typename T, int TX, int TY, int NT>
struct StageLds {
    static constexpr int RX = TX + 6, RY = TY + 6, NR = RX * RY;   // tile + 3
    static constexpr int GX = TX + 2, GY = TY + 2, NG = GX * GY;   // tile + 1
    static constexpr int NFX = (TX + 1) * TY, NFY = TX * (TY + 1);
    // the magnetic block of the sweeps run inside stage 1 (tile + a halo of 2 MAG_KMAX + 3)
    static constexpr int MRX = TX + 4 * MAG_KMAX + 6, MRY = TY + 4 * MAG_KMAX + 6;
    static constexpr int MB = MRX * MRY + MRX * MRY / 2 * 2;
    static_assert(5 * (NFX + NFY) <= (NQ + 1 - Q_P) * NR, "the fluxes fit in the dead cell fields");
    T qbuf[(NQ + 1) * NR];   // q(k) for k < NQ, then mu_c
    T fl[TX * TY];           // liquid fraction of the tile's cells (phases A-E)
    union {
        struct {
            T g[NV][2][NG];  // d/dx, d/dy of p, u, v, rho, C, mu_c, T, He (phases C-E)
            T h2[NG];        // |H|^2
        };
        double cd[NR];       // the order parameter in FP64 (phases A-B)
        T mblk[MB];          // the magnetic block (stage 1 with the sweeps, phases M-A)
    };
    __device__ T* q(int k) { return qbuf + k * NR; }
    __device__ const T* q(int k) const { return qbuf + k * NR; }
    __device__ T* muc() { return qbuf + NQ * NR; }
    __device__ T* fx(int k) { return qbuf + Q_P * NR + k * NFX; }
    __device__ T* fy(int k) { return qbuf + Q_P * NR + 5 * NFX + k * NFY; }
};

// gather one side of a face from LDS; axis 0: x-face (n = x, t = y), 1: y-face
template <typename T, typename L>
__device__ __forceinline__ void gather_side(const L& s, int r, int gidx, int axis, Side<T>& o)
{
    const int in = axis == 0 ? 0 : 1, it = 1 - in;
    o.v[V_P] = s.q(Q_P)[r];
    o.v[V_UN] = axis == 0 ? s.q(Q_U)[r] : s.q(Q_V)[r];
    o.v[V_UT] = axis == 0 ? s.q(Q_V)[r] : s.q(Q_U)[r];
    o.v[V_RHO] = s.q(Q_RHO)[r];
    o.v[V_C] = s.q(Q_C)[r];
    o.v[V_MUC] = s.qbuf[NQ * L::NR + r];
    o.v[V_T] = s.q(Q_T)[r];
    o.v[V_HE] = s.q(Q_HE)[r];
    // gradient slots: 0 p, 1 u, 2 v, 3 rho, 4 C, 5 muc, 6 T, 7 He
    const int slot[NV] = {0, axis == 0 ? 1 : 2, axis == 0 ? 2 : 1, 3, 4, 5, 6, 7};
#pragma unroll
    for (int k = 0; k < NV; k++) {
        o.gn[k] = s.g[slot[k]][in][gidx];
        o.gt[k] = s.g[slot[k]][it][gidx];
    }
    o.mu = s.q(Q_MU)[r];
    o.lam = s.q(Q_LAM)[r];
    o.cp = s.q(Q_CP)[r];
}

// the LBFS flux of face fi of one axis (AX 0: x-face, cells L = (cx-1, cy), R = (cx, cy);
// 1: y-face, L = (cx, cy-1), R = (cx, cy)) of a tile, with the wall conditions (only a
// tile with a side on the domain edge, edge != 0, has wall faces), into F (He, p, normal
// and tangential momentum, C)
template <typename T, int TX, int TY, int AX, typename L>
__device__ __forceinline__ void split_face(L& s, const Coef<T>& K, const DevInst& I, int x0, int y0, bool edge,
                                           int fi, T F[5])
{
    int cx, cy, lxL, lyL;
    if constexpr (AX == 0) {
        cx = fi % (TX + 1); cy = fi / (TX + 1);
        lxL = cx - 1; lyL = cy;
    } else {
        cx = fi % TX; cy = fi / TX;
        lxL = cx; lyL = cy - 1;
    }
    const int rL = (lyL + 3) * L::RX + (lxL + 3), rR = (cy + 3) * L::RX + (cx + 3);
    const int gL = (lyL + 1) * L::GX + (lxL + 1), gR = (cy + 1) * L::GX + (cx + 1);
    SidePart<T> PL, PR;
    {
        Side<T> S;
        gather_side<T>(s, rL, gL, AX, S);
        side_part<T, 1>(K, S, PL);
    }
    // (a compiler fence: each side's fields are read from one base address, rather than
    // each field plane of both sides from a base of its own)
    asm volatile("" ::: "memory");
    {
        Side<T> S;
        gather_side<T>(s, rR, gR, AX, S);
        side_part<T, -1>(K, S, PR);
    }
    face_flux<T>(K, PL, PR, F);
    // walls: no mass or order-parameter flux; heat through the half cell
    const int gface = AX == 0 ? x0 + cx : y0 + cy;
    const int nax = AX == 0 ? I.nx : I.ny;
    const int per = AX == 0 ? I.per_x : I.per_y;
    if (edge && !per && (gface == 0 || gface == nax)) {
        const bool lo = gface == 0;
        const int wall = AX == 0 ? (lo ? 0 : 1) : (lo ? 2 : 3);
        const int rc = lo ? rR : rL;
        F[1] = T(0);
        F[4] = T(0);
        if (I.tbc[wall]) {
            const T k = s.q(Q_LAM)[rc] * rcp_bounded(s.q(Q_RHO)[rc]);
            const T Tc = s.q(Q_T)[rc], Tw = K.tval[wall];
            F[0] = lo ? -k * (Tc - Tw) * K.i_halfdx : -k * (Tw - Tc) * K.i_halfdx;
        } else {
            F[0] = T(0);
        }
    }
}

__device__ __forceinline__ double wave_sum(double x)
{
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}
__device__ __forceinline__ double wave_max(double x)
{
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
    return x;
}

// FP64 observables of one cell of the state Wn (He, p, Mx, My, C): clamped order
// parameter, Ct Fl, Fs, |u|, non-finite flag, |u| inside the drop, height column (Ct and
// Fs), heat into a fixed south wall (-lambda dT/dy over the half cell, times dx), and the
// first and second moments of Ct about the origin (droplet centroid and axes).
template <typename T>
__device__ __forceinline__ void cell_partials(const DevInst& I, const T* Wn, double Cd, int gx, int gy, double* pr)
{
    T T1, Fl1;
    const Coef<T>& K = coef<T>(I);
    enthalpy_state<T>(K, Wn[0], T(Cd), T1, Fl1);
    const T ct1 = clamp01(T(Cd));
    const T fs1 = ct1 * (T(1) - Fl1);
    const T rho1 = mix3<T>(K.rho, fs1, ct1);
    const double ctd = clamp01(Cd);   // (the clamped order parameter of the sums in FP64)
    const double u1 = double(Wn[2]) * 3.0 / double(rho1), v1 = double(Wn[3]) * 3.0 / double(rho1);
    const double um = sqrt(u1 * u1 + v1 * v1);
    bool finite = true;
#pragma unroll
    for (int k = 0; k < 4; k++) finite = finite && isfinite(double(Wn[k]));
    finite = finite && isfinite(Cd);
    pr[PART_CT] = ctd;
    pr[PART_CTFL] = ctd * double(Fl1);
    pr[PART_FS] = ctd * (1.0 - double(Fl1));
    pr[PART_UMAX] = um;
    pr[PART_NONFINITE] = finite ? 0.0 : 1.0;
    pr[PART_UDROP] = ctd >= 0.5 ? um : 0.0;
    pr[PART_HEIGHT] = gx == I.col_height ? ctd : 0.0;
    pr[PART_SOLIDH] = gx == I.col_height ? pr[PART_FS] : 0.0;
    const double x = (gx + 0.5) * I.dx, y = (gy + 0.5) * I.dx, c = ctd;
    pr[PART_MX] = c * x;
    pr[PART_MY] = c * y;
    pr[PART_MXX] = c * x * x;
    pr[PART_MYY] = c * y * y;
    pr[PART_MXY] = c * x * y;
    pr[PART_HEAT] = 0.0;
    if (gy == 0 && I.heat_on) {
        const double lam1 = double(mix3<T>(K.lam, fs1, ct1));
        pr[PART_HEAT] = -lam1 * (double(T1) - I.tval[2]) / (0.5 * I.dx) * I.dx;
    }
}

__device__ __forceinline__ bool part_is_max(int k)
{
    return k == PART_UMAX || k == PART_NONFINITE || k == PART_UDROP;
}

// fixed-order workgroup reduction of the per-thread partials into out[NPART]
template <int NT>
__device__ __forceinline__ void block_partials(const double* pr, double (*red)[NT / 64], int tid, double* out)
{
    const int wave = tid / 64, lane = tid % 64;
#pragma unroll
    for (int k = 0; k < NPART; k++) {
        const double w = part_is_max(k) ? wave_max(pr[k]) : wave_sum(pr[k]);
        if (lane == 0) red[k][wave] = w;
    }
    __syncthreads();
    if (tid < NPART) {
        const int k = tid;
        double acc = red[k][0];
        for (int w = 1; w < NT / 64; w++) acc = part_is_max(k) ? fmax(acc, red[k][w]) : acc + red[k][w];
        out[k] = acc;
    }
}

__device__ __forceinline__ bool res_is_max(int k)
{
    return k == RES_UMAX || k == RES_NONFINITE || k == RES_UDROP;
}

// Fixed-order FP64 reduction of an instance's tile partials (and the magnetic
// residual partials) into I.result; NT threads of one workgroup.
template <int NT>
__device__ __forceinline__ void instance_reduce(const DevInst& I, int tid, double (*red)[NT / 64], int mres_stage)
{
    double acc[NRES] = {};
    for (int t = tid; t < I.ntile_stage; t += NT) {
        const double* p = I.part + (size_t)t * NPART;
        acc[RES_CT] += p[PART_CT];
        acc[RES_CTFL] += p[PART_CTFL];
        acc[RES_FS] += p[PART_FS];
        acc[RES_UMAX] = fmax(acc[RES_UMAX], p[PART_UMAX]);
        acc[RES_NONFINITE] = fmax(acc[RES_NONFINITE], p[PART_NONFINITE]);
        acc[RES_UDROP] = fmax(acc[RES_UDROP], p[PART_UDROP]);
        acc[RES_HEIGHT] += p[PART_HEIGHT];
        acc[RES_HEAT] += p[PART_HEAT];
        acc[RES_MX] += p[PART_MX];
        acc[RES_MY] += p[PART_MY];
        acc[RES_MXX] += p[PART_MXX];
        acc[RES_MYY] += p[PART_MYY];
        acc[RES_MXY] += p[PART_MXY];
        acc[RES_SOLIDH] += p[PART_SOLIDH];
    }
    const int nm = mres_stage ? I.ntile_stage : I.ntile_mag;
    for (int t = tid; t < nm; t += NT) acc[RES_MAGR2] += I.mpart[t];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NRES; k++) {
        const double w = res_is_max(k) ? wave_max(acc[k]) : wave_sum(acc[k]);
        if (tid % 64 == 0) red[k][tid / 64] = w;
    }
    __syncthreads();
    if (tid < NRES) {
        const int k = tid;
        double a = red[k][0];
        for (int w = 1; w < NT / 64; w++) a = res_is_max(k) ? fmax(a, red[k][w]) : a + red[k][w];
        I.result[k] = a;
    }
}

// NT >= every per-tile work count (halo cells, gradient cells, faces), so each phase
// is one round; the first TX*TY threads own the tile's cells. The register bound asks
// for seven 256-thread workgroups per CU in FP32 (69 VGPRs) and four in FP64 (128),
// which is what the LDS of the default tiles allows.
template <typename T, int TX, int TY, int NT, int STAGE, int EARLY, int FUSE>
__global__ __launch_bounds__(NT, NT == 256 ? (sizeof(T) == 4 ? 7 : 4) : 1) void k_stage(const DevInst* __restrict__ insts,
                                              const Tile* __restrict__ tiles, int pidx, int nsweeps, double omega)
{
    using L = StageLds<T, TX, TY, NT>;
    static_assert(NT % 64 == 0 && NT >= TX * TY, "whole waves, one thread per cell at least");
    static_assert(!FUSE || STAGE == 1, "the magnetic phase fuses into stage 1");
    __shared__ L s;
    const Tile tile = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const DevInst& I = insts[tile.inst];
    const int tid = threadIdx.x;
    const int x0 = tile.x0, y0 = tile.y0;
    const int nx = I.nx, ny = I.ny, pitch = I.pitch;
    const Coef<T>& K = coef<T>(I);
    const T dx = K.dx;
    const T inv2dx = K.inv2dx;

    // He, p, Mx, My in the instance precision; the order parameter C (index 4) is stored
    // in FP64 in both precisions
    T* const* Wbase = reinterpret_cast<T* const*>(I.W);
    T* const* Win = STAGE == 2 ? reinterpret_cast<T* const*>(I.W1)
                  : STAGE == 3 ? reinterpret_cast<T* const*>(I.W2) : Wbase;
    const GLOBAL double* Cbase = gp<double>(I.W[4]);
    const GLOBAL double* Cin = gp<double>(STAGE == 2 ? I.W1[4] : STAGE == 3 ? I.W2[4] : I.W[4]);
    const GLOBAL T* phi = gp<T>(I.phi[pidx]);

    // cell owned by this thread (phase E). With EARLY, stages 0 and 1 fetch its point
    // values now, overlapping the halo phases; otherwise they are loaded in phase E,
    // which keeps the registers free for the faces (other workgroups on the CU hide the
    // latency).
    const int lx = tid % TX, ly = tid / TX;
    const int gx = x0 + lx, gy = y0 + ly;
    const bool inside = tid < TX * TY && gx < nx && gy < ny;
    // the owned cell's element of a field: the tile origin's address (uniform, in scalar
    // registers) plus a 32-bit byte offset, so the accesses of every field share one
    // vector offset instead of a 64-bit address each
    const size_t t0 = (size_t)y0 * pitch + x0;
    const uint32_t ob = inside ? (uint32_t)(ly * pitch + lx) : 0u;
    auto own = [&](void* field) -> GLOBAL T& {
        return *(GLOBAL T*)((GLOBAL char*)(gp<T>(field) + t0) + ob * (uint32_t)sizeof(T));
    };
    auto own_d = [&](void* field) -> GLOBAL double& {
        return *(GLOBAL double*)((GLOBAL char*)(gp<double>(field) + t0) + ob * 8u);
    };
    constexpr bool early = EARLY && STAGE <= 1;
    // The Kelvin force (Eq. 6) takes chi from the step-start state and |H|^2 from the
    // step's potential, which the stages do not change: stages 0 (R(W) alone) and 1
    // compute it, stage 1 leaves it in I.kf with the step-start liquid fraction, and
    // stages 2 and 3 read them (the potential is then not loaded at all).
    constexpr bool KELVIN = STAGE <= 1;

    // ---- M (FUSE): the step's magnetic phase for this tile: red-black sweeps of the tile
    //      plus a halo of 2*MAG_KMAX+3 cells in LDS (the arithmetic of k_mag_fused, so
    //      the potential is the same bit for bit, and exact on tile + 3), written to the
    //      other potential buffer with this tile's FP64 residual partial; phase A takes
    //      the potential from LDS. The block lives in the storage of the face-phase
    //      arrays, which phases C and D fill only after A.
    constexpr int HM = 2 * MAG_KMAX + 3;
    using GM = MagGeom<TX, TY, HM>;
    T (*const mph)[GM::HALF] = reinterpret_cast<T (*)[GM::HALF]>(&s.mblk[0]);
    const int mpar0 = (x0 - HM + y0 - HM) & 1;
    auto mphi = [&](int px, int py) {   // potential of grid cell (px, py) from the block
        int lxm = px - x0 + HM, lym = py - y0 + HM;
        lxm = lxm < 0 ? 0 : (lxm >= GM::RX ? GM::RX - 1 : lxm);
        lym = lym < 0 ? 0 : (lym >= GM::RY ? GM::RY - 1 : lym);
        return mph[(mpar0 + lxm + lym) & 1][lym * GM::RXH + (lxm >> 1)];
    };
    if constexpr (FUSE) {
        static_assert(2 * GM::HALF + GM::NR <= L::MB, "the magnetic block fits in its LDS");
        __shared__ double mred[NT / 64];
        T* const mmu = &mph[0][0] + 2 * GM::HALF;
        const double r2 = mag_block<T, TX, TY, NT, HM>(I, x0, y0, pidx, nsweeps, omega, 1, mph, mmu);
        GLOBAL T* phout = gp<T>(I.phi[pidx ^ 1]);
        for (int c = tid; c < TX * TY; c += NT) {
            const int tx = c % TX, ty = c / TX;
            if (x0 + tx >= nx || y0 + ty >= ny) continue;
            phout[(size_t)(y0 + ty) * pitch + (x0 + tx)] = mphi(x0 + tx, y0 + ty);
        }
        const double w = wave_sum(r2);
        if (tid % 64 == 0) mred[tid / 64] = w;
        __syncthreads();
        if (tid == 0) {
            double acc = 0.0;
            for (int k = 0; k < NT / 64; k++) acc += mred[k];
            I.mpart[tile.idx] = acc;
        }
    }
    T cWin[4], cWb[4], cS = T(0);
    double cCin = 0.0, cCb = 0.0;
    auto load_own = [&] {
#pragma unroll
        for (int k = 0; k < 4; k++) {
            cWin[k] = STAGE >= 1 ? own(Win[k]) : T(0);
            cWb[k] = STAGE >= 2 ? own(Wbase[k]) : T(0);
        }
        cCin = STAGE >= 1 ? own_d(STAGE == 2 ? I.W1[4] : STAGE == 3 ? I.W2[4] : I.W[4]) : 0.0;
        cCb = STAGE >= 2 ? own_d(I.W[4]) : 0.0;
        cS = own(I.S);
    };
    if constexpr (early) load_own();

    // ---- A: cell fields of tile + 3 (ghosts by mirror / periodic image); every load of
    //      this thread is issued before the first one is used. A tile whose halo lies
    //      inside the domain (most of them) takes a path without images or mirrors.
    const bool interior = x0 >= 3 && y0 >= 3 && x0 + TX + 3 <= nx && y0 + TY + 3 <= ny;
    // (in FP64 the order parameter of s.q is the FP64 one: no second copy)
    constexpr bool cd_copy = sizeof(T) < sizeof(double);
    auto store_cell = [&](int r, const Prim<T>& q, T ph, double cdv) {
        if constexpr (cd_copy) s.cd[r] = cdv;
        s.q(Q_P)[r] = q.p;
        s.q(Q_U)[r] = q.u;
        s.q(Q_V)[r] = q.v;
        s.q(Q_RHO)[r] = q.rho;
        s.q(Q_C)[r] = q.C;
        s.q(Q_T)[r] = q.Tt;
        s.q(Q_HE)[r] = q.He;
        s.q(Q_MU)[r] = q.mu;
        s.q(Q_LAM)[r] = q.lam;
        s.q(Q_CP)[r] = q.cp;
        if constexpr (KELVIN) s.q(Q_PHI)[r] = ph;
        // the tile's own cells keep their liquid fraction for phase E
        const int tx = r % L::RX - 3, ty = r / L::RX - 3;
        if ((unsigned)tx < (unsigned)TX && (unsigned)ty < (unsigned)TY) s.fl[ty * TX + tx] = q.Fl;
    };
    constexpr int NIT = (L::NR + NT - 1) / NT;
    if (interior) {
        T vW[NIT][4], vph[NIT];
        double vC[NIT];
        // (addresses from the region origin (x0 - 3, y0 - 3), which lies inside the
        // domain here: a uniform base plus a 32-bit byte offset per cell)
        const size_t h0 = (size_t)(y0 - 3) * pitch + (x0 - 3);
#pragma unroll
        for (int it = 0; it < NIT; it++) {
            const int r = tid + it * NT;
            const int rr = r < L::NR ? r : L::NR - 1;
            const uint32_t oh = (uint32_t)((rr / L::RX) * pitch + rr % L::RX);
#pragma unroll
            for (int k = 0; k < 4; k++)
                vW[it][k] = *(const GLOBAL T*)((const GLOBAL char*)(gp<T>(Win[k]) + h0) + oh * (uint32_t)sizeof(T));
            vC[it] = *(const GLOBAL double*)((const GLOBAL char*)(Cin + h0) + oh * 8u);
            if constexpr (FUSE) vph[it] = mphi(x0 - 3 + rr % L::RX, y0 - 3 + rr / L::RX);
            else if constexpr (KELVIN)
                vph[it] = *(const GLOBAL T*)((const GLOBAL char*)(phi + h0) + oh * (uint32_t)sizeof(T));
            else vph[it] = T(0);
        }
        // (the FP64 order parameter shares LDS with the magnetic block of FUSE: every
        // potential is read before the first is overwritten)
        if constexpr (FUSE && cd_copy) __syncthreads();
#pragma unroll
        for (int it = 0; it < NIT; it++) {
            const int r = tid + it * NT;
            if (r >= L::NR) break;
            store_cell(r, primitives<T>(K, vW[it][0], vW[it][1], vW[it][2], vW[it][3], T(vC[it])), vph[it],
                       vC[it]);
        }
    } else {
        T vW[NIT][4], vph[NIT];
        double vC[NIT];
        int vwx[NIT], vwy[NIT], vdx[NIT], vdy[NIT];
#pragma unroll
        for (int it = 0; it < NIT; it++) {
            const int r = tid + it * NT;
            const int rr = r < L::NR ? r : L::NR - 1;
            const int hx = x0 - 3 + rr % L::RX, hy = y0 - 3 + rr / L::RX;
            int wx, wy;
            const int sx = map_axis(hx, nx, I.per_x, 0, 1, wx);
            const int sy = map_axis(hy, ny, I.per_y, 2, 3, wy);
            vwx[it] = wx;
            vwy[it] = wy;
            vdx[it] = sx - hx;
            vdy[it] = sy - hy;
            const size_t oh = (size_t)sy * pitch + sx;
#pragma unroll
            for (int k = 0; k < 4; k++) vW[it][k] = gp<T>(Win[k])[oh];
            vC[it] = Cin[oh];
            // (the block holds periodic images in place and zeros beyond walls: a wall
            // ghost reads its mirror cell)
            if constexpr (FUSE) vph[it] = mphi(wx >= 0 ? sx : hx, wy >= 0 ? sy : hy);
            else if constexpr (KELVIN) vph[it] = phi[oh];
            else vph[it] = T(0);
        }
        if constexpr (FUSE && cd_copy) __syncthreads();
#pragma unroll
        for (int it = 0; it < NIT; it++) {
            const int r = tid + it * NT;
            if (r >= L::NR) break;
            double cdv = vC[it];
            Prim<T> q = primitives<T>(K, vW[it][0], vW[it][1], vW[it][2], vW[it][3], T(cdv));
            T ph = vph[it];
            const int wx = vwx[it], wy = vwy[it];
            // a wetting wall adds the contact-angle gradient to the mirrored order
            // parameter over the |vd| cells between ghost and mirror cell (in FP64, the
            // precision of the stored order parameter)
            auto wet = [&](double c, double wk, int vd) {
                const double cc = clamp01(c);
                return c + double(vd < 0 ? -vd : vd) * I.dx * wk * cc * (1.0 - cc);
            };
            if (wx >= 0) {
                q.u = -q.u;
                q.v = -q.v;
                if (I.tbc[wx]) q.Tt = T(2) * K.tval[wx] - q.Tt;
                ph = I.mbc[wx] ? -ph : ph - K.h0x * T(vdx[it]) * dx;
                if (I.wet[wx] != 0.0) cdv = wet(cdv, I.wet[wx], vdx[it]);
            }
            if (wy >= 0) {
                q.u = -q.u;
                q.v = -q.v;
                if (I.tbc[wy]) q.Tt = T(2) * K.tval[wy] - q.Tt;
                ph = I.mbc[wy] ? -ph : ph - K.h0y * T(vdy[it]) * dx;
                if (I.wet[wy] != 0.0) cdv = wet(cdv, I.wet[wy], vdy[it]);
            }
            q.C = T(cdv);
            store_cell(r, q, ph, cdv);
        }
    }
    __syncthreads();

    // ---- B: chemical potential on tile + 2 (mu_c = 2 beta C (C-1)(2C-1) - kappa lap C),
    //      in FP64 from the FP64 order parameter: in the bulk phases mu_c is nearly
    //      zero, and the rounding of C to FP32, amplified by kappa / dx^2 in the
    //      Laplacian, would dominate it and the capillary force
    {
        const Coef<double>& KD = coef<double>(I);
        const double beta = KD.beta, kappa = KD.kappa, idx2 = KD.idx2;
        for (int r = tid; r < L::NR; r += NT) {
            const int lx = r % L::RX, ly = r / L::RX;
            if (lx < 1 || lx >= L::RX - 1 || ly < 1 || ly >= L::RY - 1) continue;
            const double* C = cd_copy ? s.cd : reinterpret_cast<const double*>(s.q(Q_C));
            const double c = C[r];
            const double lap = (C[r + 1] + C[r - 1] + C[r + L::RX] + C[r - L::RX] - 4.0 * c) * idx2;
            s.muc()[r] = T(2.0 * beta * c * (c - 1.0) * (2.0 * c - 1.0) - kappa * lap);
        }
    }
    __syncthreads();
    // wall ghosts take the chemical potential of their mirror cell (no flux of C through
    // a wall: d(mu_c)/dn = 0) when a wetting wall's ghosts are not mirrors of the order
    // parameter (otherwise the ghost values computed above are that mirror already). A
    // mirror cell is never a wall ghost, so one pass reads only cells it does not write.
    if (!interior && (K.wet[0] != T(0) || K.wet[1] != T(0) || K.wet[2] != T(0) || K.wet[3] != T(0))) {
        for (int r = tid; r < L::NR; r += NT) {
            const int lx = r % L::RX, ly = r / L::RX;
            if (lx < 1 || lx >= L::RX - 1 || ly < 1 || ly >= L::RY - 1) continue;
            const int gx = x0 - 3 + lx, gy = y0 - 3 + ly;
            const bool wallx = !I.per_x && (gx < 0 || gx >= nx);
            const bool wally = !I.per_y && (gy < 0 || gy >= ny);
            if (!wallx && !wally) continue;
            const int mx = wallx ? (gx < 0 ? -1 - gx : 2 * nx - 1 - gx) : gx;
            const int my = wally ? (gy < 0 ? -1 - gy : 2 * ny - 1 - gy) : gy;
            const int mlx = mx - (x0 - 3), mly = my - (y0 - 3);
            // (cells further than the halo from a tiny domain mirror out of the domain or
            // the region; their values never reach an output)
            if (mx < 0 || mx >= nx || my < 0 || my >= ny || mlx < 1 || mlx > L::RX - 2 || mly < 1 ||
                mly > L::RY - 2)
                continue;
            s.muc()[r] = s.muc()[mly * L::RX + mlx];
        }
        __syncthreads();
    }

    // ---- C: central gradients and |H|^2 on tile + 1
    const T h0x = K.h0x, h0y = K.h0y;
    for (int gi = tid; gi < L::NG; gi += NT) {
        const int lx = gi % L::GX + 2, ly = gi / L::GX + 2;
        const int r = ly * L::RX + lx;
        const T* src[NV] = {s.q(Q_P), s.q(Q_U), s.q(Q_V), s.q(Q_RHO), s.q(Q_C), s.muc(), s.q(Q_T), s.q(Q_HE)};
#pragma unroll
        for (int k = 0; k < NV; k++) {
            s.g[k][0][gi] = (src[k][r + 1] - src[k][r - 1]) * inv2dx;
            s.g[k][1][gi] = (src[k][r + L::RX] - src[k][r - L::RX]) * inv2dx;
        }
        const int gx = x0 - 3 + lx, gy = y0 - 3 + ly;
        const bool wallx = !interior && !I.per_x && (gx < 0 || gx >= nx);
        const bool wally = !interior && !I.per_y && (gy < 0 || gy >= ny);
        if (KELVIN && !wallx && !wally) {
            const T* P = s.q(Q_PHI);
            const T Hx = h0x - (P[r + 1] - P[r - 1]) * inv2dx;
            const T Hy = h0y - (P[r + L::RX] - P[r - L::RX]) * inv2dx;
            s.h2[gi] = Hx * Hx + Hy * Hy;
        }
    }
    __syncthreads();
    // |H|^2 of wall ghosts mirrors the interior cell (no wall ghosts on interior tiles)
    for (int gi = tid; gi < (interior || !KELVIN ? 0 : L::NG); gi += NT) {
        const int lx = gi % L::GX + 2, ly = gi / L::GX + 2;
        const int gx = x0 - 3 + lx, gy = y0 - 3 + ly;
        const bool wallx = !I.per_x && (gx < 0 || gx >= nx);
        const bool wally = !I.per_y && (gy < 0 || gy >= ny);
        if (!wallx && !wally) continue;
        int mx = gx, my = gy;
        if (wallx) mx = gx < 0 ? -1 - gx : 2 * nx - 1 - gx;
        if (wally) my = gy < 0 ? -1 - gy : 2 * ny - 1 - gy;
        int mlx = mx - (x0 - 3) - 2, mly = my - (y0 - 3) - 2;
        mlx = mlx < 0 ? 0 : (mlx >= L::GX ? L::GX - 1 : mlx);
        mly = mly < 0 ? 0 : (mly >= L::GY ? L::GY - 1 : mly);
        const int mg = mly * L::GX + mlx;
        const bool mwx = !I.per_x && (mx < 0 || mx >= nx);
        const bool mwy = !I.per_y && (my < 0 || my >= ny);
        s.h2[gi] = (mwx || mwy) ? T(0) : s.h2[mg];
    }

    // ---- D: LBFS fluxes of all faces of the tile: x-faces on the first NXT threads,
    //      y-faces on the next NYT (whole waves each), so the axis is the same on every lane
    //      of a wave and the LDS offsets and the component swap are constants. Every face
    //      of every tile shape goes through the same two instantiations of the flux.
    //      The fluxes stay in registers until every face has read its cells, then take
    //      the place of the cell fields that are dead from here on. Lanes past an axis's
    //      last face repeat that face (no masked lanes in the flux); they store nothing.
    {
        const bool edge = x0 == 0 || y0 == 0 || x0 + TX >= nx || y0 + TY >= ny;
        constexpr int NXT = (L::NFX + 63) / 64 * 64, NYT = (L::NFY + 63) / 64 * 64;
        constexpr int NRND = (NXT + NYT + NT - 1) / NT;
        T Fr[NRND][5];
#pragma unroll
        for (int k = 0; k < NRND; k++) {
            const int f = tid + k * NT;
            if (f >= NXT + NYT) break;
            if (__builtin_amdgcn_readfirstlane(f) < NXT) {
                split_face<T, TX, TY, 0>(s, K, I, x0, y0, edge, f < L::NFX ? f : L::NFX - 1, Fr[k]);
            } else {
                split_face<T, TX, TY, 1>(s, K, I, x0, y0, edge, f - NXT < L::NFY ? f - NXT : L::NFY - 1, Fr[k]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NRND; k++) {
            const int f = tid + k * NT;
            if (f >= NXT + NYT) break;
            const T* F = Fr[k];
            if (f < NXT) {
                if (f < L::NFX) {
                    s.fx(0)[f] = F[0]; s.fx(1)[f] = F[1]; s.fx(2)[f] = F[2]; s.fx(3)[f] = F[3]; s.fx(4)[f] = F[4];
                }
            } else if (f - NXT < L::NFY) {
                const int fi = f - NXT;
                s.fy(0)[fi] = F[0]; s.fy(1)[fi] = F[1]; s.fy(2)[fi] = F[3]; s.fy(3)[fi] = F[2]; s.fy(4)[fi] = F[4];
            }
        }
    }
    __syncthreads();

    // ---- E: residual, sources, Runge-Kutta stage
    if (inside) {
        if constexpr (!early) load_own();
        const int r = (ly + 3) * L::RX + (lx + 3);
        const int gi = (ly + 1) * L::GX + (lx + 1);
        const T dt = K.dt;
        const T idt = K.idt, idx = K.idx;
        const T cs2 = T(1.0 / 3.0);
        // the liquid fraction of this stage's state, from phase A (stages 0 and 1 take
        // the step-start state)
        const T Flc = s.fl[tid];
        // Kelvin force from the step-start state (Eq. 6)
        T fmx, fmy, Fln;
        if constexpr (KELVIN) {
            const T Cn = s.q(Q_C)[r];
            Fln = Flc;
            const T ctn = clamp01(Cn);
            const T chi = mix3<T>(K.chi, ctn * (T(1) - Fln), ctn);
            const T kmg = T(0.5) * K.mu0 * chi;
            fmx = kmg * (s.h2[gi + 1] - s.h2[gi - 1]) * inv2dx;
            fmy = kmg * (s.h2[gi + L::GX] - s.h2[gi - L::GX]) * inv2dx;
            if constexpr (STAGE == 1) {
                own(I.kf[0]) = fmx;
                own(I.kf[1]) = fmy;
                own(I.kf[2]) = Fln;
            }
        } else {
            fmx = own(I.kf[0]);
            fmy = own(I.kf[1]);
            Fln = STAGE == 3 ? own(I.kf[2]) : T(0);
        }
        // stage-state cell fields; the central gradients phase C left in LDS
        const T divu = s.g[1][0][gi] + s.g[2][1][gi];
        const T drx = s.g[3][0][gi], dry = s.g[3][1][gi];
        const T dmx = s.g[5][0][gi], dmy = s.g[5][1][gi];
        const T c = s.q(Q_C)[r], rho = s.q(Q_RHO)[r], u = s.q(Q_U)[r], v = s.q(Q_V)[r];
        const T fs = clamp01(c) * (T(1) - Flc);
        const T Sv = cS;
        const T vc = K.vc;
        T src[5];
        src[0] = s.q(Q_CP)[r] * s.q(Q_T)[r] * divu;
        src[1] = cs2 * (u * drx + v * dry) + rho * cs2 * vc * Sv;
        src[2] = cs2 * (-c * dmx + fmx + rho * K.grav[0] - rho * u * fs * idt);
        src[3] = cs2 * (-c * dmy + fmy + rho * K.grav[1] - rho * v * fs * idt);
        src[4] = c * vc * Sv;
        const int fW = ly * (TX + 1) + lx, fS = ly * TX + lx;
        T Rk[5];
#pragma unroll
        for (int k = 0; k < 5; k++) {
            const T div = (s.fx(k)[fW + 1] - s.fx(k)[fW] + s.fy(k)[fS + TX] - s.fy(k)[fS]) * idx;
            Rk[k] = -div + src[k];
        }
        // (the order parameter is combined in FP64: its increment dt R_C is small)
        const double dRc = double(dt) * double(Rk[4]);
        if (STAGE == 0) {
#pragma unroll
            for (int k = 0; k < 4; k++) own(I.W1[k]) = Rk[k];
            own_d(I.W1[4]) = double(Rk[4]);
        } else if (STAGE == 1) {
#pragma unroll
            for (int k = 0; k < 4; k++) own(I.W1[k]) = cWin[k] + dt * Rk[k];
            own_d(I.W1[4]) = cCin + dRc;
        } else if (STAGE == 2) {
#pragma unroll
            for (int k = 0; k < 4; k++) own(I.W2[k]) = T(0.75) * cWb[k] + T(0.25) * (cWin[k] + dt * Rk[k]);
            own_d(I.W2[4]) = 0.75 * cCb + 0.25 * (cCin + dRc);
        } else {
            T Wn[4];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                Wn[k] = cWb[k] * T(1.0 / 3.0) + T(2.0 / 3.0) * (cWin[k] + dt * Rk[k]);
                own(Wbase[k]) = Wn[k];
            }
            const double Cn1 = cCb * (1.0 / 3.0) + (2.0 / 3.0) * (cCin + dRc);
            own_d(I.W[4]) = Cn1;
            // Table 1 (d): Eq. 8 after the step; lagged dFs/dt for the next step
            T T1, Fl1;
            enthalpy_state<T>(K, Wn[0], T(Cn1), T1, Fl1);
            const T ct1 = clamp01(T(Cn1));
            own(I.S) = -ct1 * (Fl1 - Fln) * idt;
            // the permeability of the new state, for the next step's magnetic phase (in
            // the Kelvin-force field, which stage 1 of that step rewrites after it)
            own(I.kf[0]) = mag_permeability<T>(K, ct1, Fl1);
        }
    }
}

// stage 4 is stage 1 with the magnetic phase fused in front of it
template <typename T, int TX, int TY, int NT, int EARLY>
hipError_t launch_stage_shape(int stage, int pidx, int nsw, double om, const DevInst* insts, const Tile* tiles,
                              int ntiles, hipStream_t stream, hipEvent_t e0, hipEvent_t e1)
{
    const dim3 grid(ntiles), block(NT);
    switch (stage) {
    case 0:
        return launch_timed(k_stage<T, TX, TY, NT, 0, EARLY, 0>, grid, block, stream, e0, e1, insts, tiles, pidx, nsw, om);
    case 1:
        return launch_timed(k_stage<T, TX, TY, NT, 1, EARLY, 0>, grid, block, stream, e0, e1, insts, tiles, pidx, nsw, om);
    case 2:
        return launch_timed(k_stage<T, TX, TY, NT, 2, 0, 0>, grid, block, stream, e0, e1, insts, tiles, pidx, nsw, om);
    case 3:
        return launch_timed(k_stage<T, TX, TY, NT, 3, 0, 0>, grid, block, stream, e0, e1, insts, tiles, pidx, nsw, om);
    default:
        return launch_timed(k_stage<T, TX, TY, NT, 1, EARLY, 1>, grid, block, stream, e0, e1, insts, tiles, pidx, nsw, om);
    }
}

// dispatch a run-time shape index to the kernel instantiated for that table entry
template <typename T, int K>
hipError_t launch_stage_idx(int shape, int stage, int pidx, int nsw, double om, const DevInst* insts,
                            const Tile* tiles, int ntiles, hipStream_t stream, hipEvent_t e0, hipEvent_t e1)
{
    if constexpr (K < NSTAGE_SHAPES) {
        constexpr TileShape S = stage_shape(sizeof(T) == 8, K);
        if (shape == K)
            return launch_stage_shape<T, S.tx, S.ty, S.nt, S.early>(stage, pidx, nsw, om, insts, tiles, ntiles,
                                                                    stream, e0, e1);
        return launch_stage_idx<T, K + 1>(shape, stage, pidx, nsw, om, insts, tiles, ntiles, stream, e0, e1);
    } else {
        return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_stage(int shape, int stage, int pidx, const DevInst* insts, const Tile* tiles, int ntiles,
                        hipStream_t stream, hipEvent_t e0, hipEvent_t e1)
{
    if (ntiles <= 0) return hipSuccess;
    if (stage < 0 || stage > 3) return hipErrorInvalidValue;
    return launch_stage_idx<T, 0>(shape, stage, pidx, 0, 1.0, insts, tiles, ntiles, stream, e0, e1);
}

template <typename T>
hipError_t launch_stage_fused(int shape, int pidx, int nsweeps, double omega, const DevInst* insts,
                              const Tile* tiles, int ntiles, hipStream_t stream, hipEvent_t e0, hipEvent_t e1)
{
    if (ntiles <= 0) return hipSuccess;
    if (nsweeps < 0 || nsweeps > MAG_KMAX) return hipErrorInvalidValue;
    return launch_stage_idx<T, 0>(shape, 4, pidx, nsweeps, omega, insts, tiles, ntiles, stream, e0, e1);
}

template <typename T>
__global__ __launch_bounds__(256) void k_state_partials(const DevInst* __restrict__ insts,
                                                        const Tile* __restrict__ tiles, int TX, int TY)
{
    __shared__ double red[NPART][4];
    const Tile tile = tiles[blockIdx.x];
    const DevInst& I = insts[tile.inst];
    double pr[NPART] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int c = threadIdx.x; c < TX * TY; c += 256) {
        const int gx = tile.x0 + c % TX, gy = tile.y0 + c / TX;
        if (gx >= I.nx || gy >= I.ny) continue;
        const size_t o = (size_t)gy * I.pitch + gx;
        T Wn[4];
#pragma unroll
        for (int k = 0; k < 4; k++) Wn[k] = reinterpret_cast<const T*>(I.W[k])[o];
        double q[NPART];
        cell_partials<T>(I, Wn, reinterpret_cast<const double*>(I.W[4])[o], gx, gy, q);
#pragma unroll
        for (int k = 0; k < NPART; k++) pr[k] = part_is_max(k) ? fmax(pr[k], q[k]) : pr[k] + q[k];
    }
    block_partials<256>(pr, red, threadIdx.x, I.part + (size_t)tile.idx * NPART);
}

template <typename T>
hipError_t launch_state_partials(int shape, const DevInst* insts, const Tile* tiles, int ntiles, hipStream_t stream)
{
    if (ntiles <= 0) return hipSuccess;
    if (shape < 0 || shape >= NSTAGE_SHAPES) return hipErrorInvalidValue;
    const TileShape S = stage_shape(sizeof(T) == 8, shape);
    hipLaunchKernelGGL((k_state_partials<T>), dim3(ntiles), dim3(256), 0, stream, insts, tiles, S.tx, S.ty);
    return hipGetLastError();
}

// ------------------------------------------------------------- magnetic kernels

// Fused magnetic phase on one tile of MTX x MTY cells: permeability (Eq. 2 with
// Eq. 11) of the tile plus a halo of 2*MAG_KMAX+1 cells, up to MAG_KMAX red-black
// sweeps of the compact system done in LDS (temporal blocking: the region where the
// sweeps are exact shrinks by one cell per colour pass), the tile's potential written
// back, and optionally the FP64 residual of the tile. Each cell update is the same
// arithmetic as an untiled red-black pass, so the result does not depend on the tiling.
//
// Update of cell c: phi'_c <- (1-w) phi'_c + w sum_f a_f (phi'_nb + phi0_nb - phi0_c) / sum_f a_f,
// a_f = mean(mu) on interior faces, 2 mu_c towards a fixed-potential wall half a cell
// away (where phi' = 0), no term at an insulating wall; phi0 = -(h0x x + h0y y).
//
// LDS holds the potential split by colour: cell (lx, ly) of colour c lives at
// ph[c][ly * RXH + lx / 2], so the cells a colour pass updates, and the neighbours it
// reads (all of the other colour), are contiguous. Each thread owns fixed cells of
// both colours and keeps their face weights, constant term and 1 / sum of weights in
// registers; a pass costs four LDS reads and one write per cell.
// A converged instance's magnetic launch: the tile's potential copied unchanged from
// buffer pin to the other one.
template <typename T, int MTX, int MTY, int NT>
__device__ __forceinline__ void copy_tile(const DevInst& I, const Tile& tile, int pin)
{
    const GLOBAL T* src = gp<T>(I.phi[pin]);
    GLOBAL T* dst = gp<T>(I.phi[pin ^ 1]);
    for (int c = threadIdx.x; c < MTX * MTY; c += NT) {
        const int gx = tile.x0 + c % MTX, gy = tile.y0 + c / MTX;
        if (gx >= I.nx || gy >= I.ny) continue;
        const size_t o = (size_t)gy * I.pitch + gx;
        dst[o] = src[o];
    }
}

// Convergence flag of one instance for the convergence-controlled magnetic phase:
// the fixed-order FP64 sum of its residual partials against mag_tol^2, stored after
// the partials (mpart[ntile_mag]).
__global__ __launch_bounds__(256) void k_mag_gate(const DevInst* __restrict__ insts)
{
    __shared__ double red[4];
    const DevInst& I = insts[blockIdx.x];
    const int tid = threadIdx.x;
    double acc = 0.0;
    for (int t = tid; t < I.ntile_mag; t += 256) acc += I.mpart[t];
    acc = wave_sum(acc);
    if (tid % 64 == 0) red[tid / 64] = acc;
    __syncthreads();
    if (tid == 0) {
        const double r2 = red[0] + red[1] + red[2] + red[3];
        I.mpart[I.ntile_mag] = r2 <= I.mag_tol * I.mag_tol ? 1.0 : 0.0;
    }
}

hipError_t launch_mag_gate(const DevInst* insts, int ninst, hipStream_t stream)
{
    if (ninst <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mag_gate, dim3(ninst), dim3(256), 0, stream, insts);
    return hipGetLastError();
}

// The halo: after nsweeps <= MAG_KMAX sweeps the cells at least 2 nsweeps from the
// region edge are exact, so a halo of 2 MAG_KMAX keeps the tile exact and one more ring
// keeps its neighbours exact for the residual (RES = 1).
template <typename T, int MTX, int MTY, int RES>
struct MagLds {
    using G = MagGeom<MTX, MTY, 2 * MAG_KMAX + RES>;
    T ph[2][G::HALF];   // potential by colour
    T mu[G::NR];        // permeability, natural layout (set-up only); 0 outside the domain
    double red[16];
};

template <typename T, int MTX, int MTY, int NT, int RES, int MUIN>
__global__ __launch_bounds__(NT) void k_mag_fused(const DevInst* __restrict__ insts,
                                                  const Tile* __restrict__ tiles, int nsweeps, double omega,
                                                  int pin, int gate)
{
    using L = MagLds<T, MTX, MTY, RES>;
    using G = typename L::G;
    static_assert(NT % 64 == 0 && NT / 64 <= 16, "whole waves");
    __shared__ L s;
    const Tile tile = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const DevInst& I = insts[tile.inst];
    if (gate && I.mpart[I.ntile_mag] != 0.0) {
        copy_tile<T, MTX, MTY, NT>(I, tile, pin);
        return;
    }
    const double r2 =
        mag_block<T, MTX, MTY, NT, G::H, MUIN>(I, tile.x0, tile.y0, pin, nsweeps, omega, RES, s.ph, s.mu);
    // write the tile in natural order (coalesced)
    GLOBAL T* phout = gp<T>(I.phi[pin ^ 1]);
    const int par0 = (tile.x0 - G::H + tile.y0 - G::H) & 1;
    for (int cidx = threadIdx.x; cidx < MTX * MTY; cidx += NT) {
        const int tx = cidx % MTX, ty = cidx / MTX;
        const int gx = tile.x0 + tx, gy = tile.y0 + ty;
        if (gx >= I.nx || gy >= I.ny) continue;
        const int lx = tx + G::H, ly = ty + G::H;
        phout[(size_t)gy * I.pitch + gx] = s.ph[(par0 + lx + ly) & 1][ly * G::RXH + (lx >> 1)];
    }
    if constexpr (RES) {
        const double w = wave_sum(r2);
        if (threadIdx.x % 64 == 0) s.red[threadIdx.x / 64] = w;
        __syncthreads();
        if (threadIdx.x == 0) {
            double acc = 0.0;
            for (int k = 0; k < NT / 64; k++) acc += s.red[k];
            I.mpart[tile.idx] = acc;
        }
    }
}

// Magnetic LBFS pseudo-time solve on one tile of MTX x MTY cells: permeability of the
// tile plus a halo of 3*RK_KMAX+1 cells, up to RK_KMAX SSP-RK3 steps of Eq. 17 done in
// LDS, the tile's potential written back, and optionally the FP64 residual. At
// delta_t = dx/2 the m* moment of Eqs. 13, 16 and 44 through a face is
// -D mu_f (phi_R - phi_L) / dx, so the rate of cell c is
// kdt (b_c + sum_f a_f phi'_nb - sum_f a_f phi'_c), kdt = D dtau / dx^2, with the face
// weights a_f and constant b_c of the sweeps (same fixed point). Each stage reads the
// previous stage's values of a cell and its four neighbours, so the exact region
// shrinks by one cell per stage; the halo keeps the tile and its neighbours (for the
// residual) exact. Every cell update is the same arithmetic whatever the tiling.
//
// LDS holds the stage values in natural layout, ping-pong between two arrays (the
// second holds the permeability during set-up). Each thread owns the region cells
// tid + j * NT and keeps their weights, constant term, pseudo-step base and current
// value in registers; a stage costs four LDS reads and one write per cell.
template <typename T, int MTX, int MTY>
struct RkLds {
    static constexpr int H = 3 * RK_KMAX + 1;
    static constexpr int RX = MTX + 2 * H, RY = MTY + 2 * H, NR = RX * RY;
    T ph[2][NR];
    double red[16];
};

template <typename T, int MTX, int MTY, int NT>
__global__ __launch_bounds__(NT) void k_mag_lbfs(const DevInst* __restrict__ insts, const Tile* __restrict__ tiles,
                                                 int nsteps, int residual, int pin, int gate)
{
    using L = RkLds<T, MTX, MTY>;
    static_assert(NT % 64 == 0 && NT / 64 <= 16, "whole waves");
    constexpr int NIT = (L::NR + NT - 1) / NT;   // owned region cells per thread
    __shared__ L s;
    const Tile tile = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const DevInst& I = insts[tile.inst];
    if (gate && I.mpart[I.ntile_mag] != 0.0) {
        copy_tile<T, MTX, MTY, NT>(I, tile, pin);
        return;
    }
    const Coef<T>& K = coef<T>(I);
    const int tid = threadIdx.x;
    const int nx = I.nx, ny = I.ny;
    const int ox = tile.x0 - L::H, oy = tile.y0 - L::H;
    const GLOBAL T* phin = gp<T>(I.phi[pin]);
    const GLOBAL T* He_ = gp<T>(I.W[0]);
    const GLOBAL double* C_ = gp<double>(I.W[4]);
    T cq[NIT];   // current value of each owned cell
    // 1. load the region: potential into ph[0], permeability into ph[1] (0 outside the
    //    domain, where the potential is 0 too)
    {
        T vHe[NIT], vC[NIT];
        bool vin[NIT];
#pragma unroll
        for (int it = 0; it < NIT; it++) {
            const int r = tid + it * NT;
            const int gx = ox + r % L::RX, gy = oy + r / L::RX;
            int sx = gx, sy = gy;
            bool in = r < L::NR;
            if (gx < 0 || gx >= nx) {
                if (I.per_x) sx = ((gx % nx) + nx) % nx;
                else in = false;
            }
            if (gy < 0 || gy >= ny) {
                if (I.per_y) sy = ((gy % ny) + ny) % ny;
                else in = false;
            }
            in = in && sx >= 0 && sx < nx && sy >= 0 && sy < ny;
            vin[it] = in;
            const size_t o = in ? (size_t)sy * I.pitch + sx : 0;
            vHe[it] = He_[o];
            vC[it] = T(C_[o]);
            cq[it] = phin[o];
        }
#pragma unroll
        for (int it = 0; it < NIT; it++) {
            const int r = tid + it * NT;
            if (r >= L::NR) break;
            T mu = T(0);
            if (vin[it]) {
                T Tt, Fl;
                enthalpy_state<T>(K, vHe[it], vC[it], Tt, Fl);
                mu = mag_permeability<T>(K, clamp01(vC[it]), Fl);
            } else {
                cq[it] = T(0);
            }
            s.ph[0][r] = cq[it];
            s.ph[1][r] = mu;
        }
    }
    __syncthreads();
    // 2. owned cells: face weights (W, E, S, N), constant part b and sum of weights d;
    //    d = 0 marks a cell that is not updated (region ring 0 or outside the domain)
    const T hx = K.h0x * K.dx, hy = K.h0y * K.dx;
    T wq[NIT][4], bq[NIT], dq[NIT], uq[NIT];
#pragma unroll
    for (int it = 0; it < NIT; it++) {
        const int r = tid + it * NT;
        bq[it] = T(0);
        dq[it] = T(0);
        uq[it] = cq[it];
#pragma unroll
        for (int d = 0; d < 4; d++) wq[it][d] = T(0);
        if (r >= L::NR) continue;
        const int lx = r % L::RX, ly = r / L::RX;
        if (lx < 1 || lx >= L::RX - 1 || ly < 1 || ly >= L::RY - 1) continue;
        const T* mu = s.ph[1];
        const T muc = mu[r];
        if (!(muc > T(0))) continue;
        const T mnb[4] = {mu[r - 1], mu[r + 1], mu[r - L::RX], mu[r + L::RX]};
        const T D0[4] = {hx, -hx, hy, -hy};   // phi0_nb - phi0_c across each face
        T bsum = T(0), den = T(0);
#pragma unroll
        for (int d = 0; d < 4; d++) {
            const bool nb_in = mnb[d] > T(0);
            const T w = nb_in ? (d == 0 || d == 2 ? T(0.5) * (mnb[d] + muc) : T(0.5) * (muc + mnb[d])) : T(0);
            wq[it][d] = w;
            if (w > T(0)) {
                bsum += w * D0[d];
                den += w;
            } else if (!nb_in && I.mbc[d]) {   // a wall face
                const T ww = T(2) * muc;
                bsum += ww * (T(0.5) * D0[d]);
                den += ww;
            }
        }
        bq[it] = bsum;
        dq[it] = den;
    }
    __syncthreads();   // the permeability in ph[1] is read by now
    // 3. SSP-RK3 in pseudo-time: stage k writes a0 u + a1 (v + kdt R(v)) into the other
    //    array, v the previous stage's values and u those at the start of the pseudo-step
    const T kdt = K.mag_kdt;
    int cur = 0;
    auto stage = [&](auto a0c, auto a1c) {
        const T a0 = T(decltype(a0c)::num) / T(decltype(a0c)::den);
        const T a1 = T(decltype(a1c)::num) / T(decltype(a1c)::den);
        const T* p = s.ph[cur];
        T* q = s.ph[cur ^ 1];
#pragma unroll
        for (int it = 0; it < NIT; it++) {
            const int r = tid + it * NT;
            if (r >= L::NR) break;
            if (dq[it] != T(0)) {
                const T rate = bq[it] + wq[it][0] * p[r - 1] + wq[it][1] * p[r + 1] + wq[it][2] * p[r - L::RX] +
                               wq[it][3] * p[r + L::RX] - dq[it] * cq[it];
                const T v = cq[it] + kdt * rate;
                cq[it] = a0 == T(0) ? v : a0 * uq[it] + a1 * v;
            }
            q[r] = cq[it];
        }
        __syncthreads();
        cur ^= 1;
    };
    using Z = std::ratio<0, 1>;
    using One = std::ratio<1, 1>;
    for (int n = 0; n < nsteps; n++) {
        stage(Z{}, One{});
        stage(std::ratio<3, 4>{}, std::ratio<1, 4>{});
        stage(std::ratio<1, 3>{}, std::ratio<2, 3>{});
#pragma unroll
        for (int it = 0; it < NIT; it++) uq[it] = cq[it];
    }
    // 4. FP64 residual r_c = b_c + sum_f a_f (phi'_nb - phi'_c) over the owned tile cells
    const T* p = s.ph[cur];
    double r2 = 0.0;
    if (residual) {
#pragma unroll
        for (int it = 0; it < NIT; it++) {
            const int r = tid + it * NT;
            if (r >= L::NR || dq[it] == T(0)) continue;
            const int tx = r % L::RX - L::H, ty = r / L::RX - L::H;
            if (tx < 0 || tx >= MTX || ty < 0 || ty >= MTY || tile.x0 + tx >= nx || tile.y0 + ty >= ny) continue;
            const double res = double(bq[it]) + double(wq[it][0]) * double(p[r - 1]) +
                               double(wq[it][1]) * double(p[r + 1]) + double(wq[it][2]) * double(p[r - L::RX]) +
                               double(wq[it][3]) * double(p[r + L::RX]) - double(dq[it]) * double(cq[it]);
            r2 += res * res;
        }
    }
    // 5. write the tile (coalesced rows)
    GLOBAL T* phout = gp<T>(I.phi[pin ^ 1]);
    for (int cidx = tid; cidx < MTX * MTY; cidx += NT) {
        const int tx = cidx % MTX, ty = cidx / MTX;
        const int gx = tile.x0 + tx, gy = tile.y0 + ty;
        if (gx >= nx || gy >= ny) continue;
        phout[(size_t)gy * I.pitch + gx] = p[(ty + L::H) * L::RX + tx + L::H];
    }
    if (residual) {
        r2 = wave_sum(r2);
        if (tid % 64 == 0) s.red[tid / 64] = r2;
        __syncthreads();
        if (tid == 0) {
            double acc = 0.0;
            for (int w = 0; w < NT / 64; w++) acc += s.red[w];
            I.mpart[tile.idx] = acc;
        }
    }
}

template <typename T, int K>
hipError_t launch_mag_lbfs_idx(int shape, const DevInst* insts, const Tile* tiles, int ntiles, hipStream_t stream,
                               hipEvent_t e0, hipEvent_t e1, int nsteps, int res, int pin, int gate)
{
    if constexpr (K < NMAG_SHAPES) {
        constexpr TileShape M = MAG_SHAPES[K];
        if (shape == K)
            return launch_timed(k_mag_lbfs<T, M.tx, M.ty, M.nt>, dim3(ntiles), dim3(M.nt), stream, e0, e1, insts,
                                tiles, nsteps, res, pin, gate);
        return launch_mag_lbfs_idx<T, K + 1>(shape, insts, tiles, ntiles, stream, e0, e1, nsteps, res, pin, gate);
    } else {
        return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_mag_lbfs(int shape, int nsteps, int residual, int* pidx, const DevInst* insts, const Tile* tiles,
                           int ntiles, hipStream_t stream, hipEvent_t e0, hipEvent_t e1, int gate)
{
    if (ntiles <= 0) return hipSuccess;
    if (shape < 0 || shape >= NMAG_SHAPES || nsteps < 0) return hipErrorInvalidValue;
    // pseudo-steps beyond the LDS halo run as further launches (timing: start of the
    // first, end of the last); each launch flips the potential buffer
    bool first = true;
    do {
        const int k = nsteps > RK_KMAX ? RK_KMAX : nsteps;
        nsteps -= k;
        const int res = residual && nsteps == 0;
        const hipEvent_t a = first ? e0 : nullptr, b = nsteps == 0 ? e1 : nullptr;
        const hipError_t e =
            launch_mag_lbfs_idx<T, 0>(shape, insts, tiles, ntiles, stream, a, b, k, res, *pidx, gate);
        if (e != hipSuccess) return e;
        *pidx ^= 1;
        first = false;
    } while (nsteps > 0);
    return hipSuccess;
}

// one launch of the fused magnetic kernel on tiles of MAG_SHAPES[shape]; res: with the
// residual (and its halo ring), muin: the permeability read from the Kelvin-force field
template <typename T, int K>
hipError_t launch_mag_idx(int shape, const DevInst* insts, const Tile* tiles, int ntiles, hipStream_t stream,
                          hipEvent_t e0, hipEvent_t e1, int nsweeps, double omega, int res, int muin, int pin,
                          int gate)
{
    if constexpr (K < NMAG_SHAPES) {
        constexpr TileShape M = MAG_SHAPES[K];
        if (shape == K) {
            const dim3 g(ntiles), b(M.nt);
            if (res)
                return muin ? launch_timed(k_mag_fused<T, M.tx, M.ty, M.nt, 1, 1>, g, b, stream, e0, e1, insts, tiles,
                                           nsweeps, omega, pin, gate)
                            : launch_timed(k_mag_fused<T, M.tx, M.ty, M.nt, 1, 0>, g, b, stream, e0, e1, insts, tiles,
                                           nsweeps, omega, pin, gate);
            return muin ? launch_timed(k_mag_fused<T, M.tx, M.ty, M.nt, 0, 1>, g, b, stream, e0, e1, insts, tiles,
                                       nsweeps, omega, pin, gate)
                        : launch_timed(k_mag_fused<T, M.tx, M.ty, M.nt, 0, 0>, g, b, stream, e0, e1, insts, tiles,
                                       nsweeps, omega, pin, gate);
        }
        return launch_mag_idx<T, K + 1>(shape, insts, tiles, ntiles, stream, e0, e1, nsweeps, omega, res, muin, pin,
                                        gate);
    } else {
        return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_mag(int shape, int nsweeps, double omega, int residual, int muin, int* pidx, const DevInst* insts,
                      const Tile* tiles, int ntiles, hipStream_t stream, hipEvent_t e0, hipEvent_t e1, int gate)
{
    if (ntiles <= 0) return hipSuccess;
    if (shape < 0 || shape >= NMAG_SHAPES) return hipErrorInvalidValue;
    // the potential is read from phi[*pidx] and written to the other buffer (halo cells
    // of a tile belong to other workgroups); sweeps beyond the LDS halo run as further
    // launches (timing: start of the first, end of the last)
    bool first = true;
    do {
        const int k = nsweeps > MAG_KMAX ? MAG_KMAX : nsweeps;
        nsweeps -= k;
        const int res = residual && nsweeps == 0;
        const hipEvent_t a = first ? e0 : nullptr, b = nsweeps == 0 ? e1 : nullptr;
        const hipError_t e =
            launch_mag_idx<T, 0>(shape, insts, tiles, ntiles, stream, a, b, k, omega, res, muin, *pidx, gate);
        if (e != hipSuccess) return e;
        *pidx ^= 1;
        first = false;
    } while (nsweeps > 0);
    return hipSuccess;
}

// ------------------------------------------------------------- reduction

__global__ __launch_bounds__(256) void k_reduce(const DevInst* __restrict__ insts, int mres_stage)
{
    __shared__ double red[NRES][4];
    instance_reduce<256>(insts[blockIdx.x], threadIdx.x, red, mres_stage);
}

hipError_t launch_reduce(const DevInst* insts, int ninst, hipStream_t stream, int mres_stage)
{
    if (ninst <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce, dim3(ninst), dim3(256), 0, stream, insts, mres_stage);
    return hipGetLastError();
}

// ------------------------------------------------------------- init / derived

// Initial fields: order parameter (tanh droplet of width xi, Fig. 8, or uniform), the
// enthalpy of temperature t_init by the inverse of Eq. 8, fluid at rest, potential of
// the applied field (phi' = 0), no lagged source.
template <typename T>
__global__ __launch_bounds__(PT_TX* PT_TY) void k_init_fields(const DevInst* __restrict__ insts,
                                                               const Tile* __restrict__ tiles,
                                                               int kind, double c_init, double t_init,
                                                               double cx, double cy, double rad)
{
    const Tile tile = tiles[blockIdx.x];
    const DevInst& I = insts[tile.inst];
    const int gx = tile.x0 + (int)threadIdx.x % PT_TX, gy = tile.y0 + (int)threadIdx.x / PT_TX;
    if (gx >= I.nx || gy >= I.ny) return;
    const size_t o = (size_t)gy * I.pitch + gx;
    const double x = (gx + 0.5) * I.dx, y = (gy + 0.5) * I.dx;
    double C = c_init;
    if (kind == 0) {
        const double r = sqrt((x - cx) * (x - cx) + (y - cy) * (y - cy));
        C = 0.5 * (1.0 + tanh(2.0 * (rad - r) / I.xi));
    }
    const double ct = C < 0.0 ? 0.0 : (C > 1.0 ? 1.0 : C);
    const double cps = ct * I.cp[0] + (1.0 - ct) * I.cp[2];
    const double cpl = ct * I.cp[1] + (1.0 - ct) * I.cp[2];
    // Eq. 8 inverted at T_init (the mushy branch only when Ts < Tl)
    const double Hes = cps * I.tm, Hel = cpl * I.tl + ct * I.latent;
    const double He = t_init >= I.tl ? cpl * t_init + ct * I.latent
                    : t_init >= I.tm ? Hes + (t_init - I.tm) / (I.tl - I.tm) * (Hel - Hes)
                                     : cps * t_init;
    reinterpret_cast<T*>(I.W[0])[o] = T(He);
    reinterpret_cast<T*>(I.W[1])[o] = T(0);
    reinterpret_cast<T*>(I.W[2])[o] = T(0);
    reinterpret_cast<T*>(I.W[3])[o] = T(0);
    reinterpret_cast<double*>(I.W[4])[o] = C;
    reinterpret_cast<T*>(I.S)[o] = T(0);
    reinterpret_cast<T*>(I.phi[0])[o] = T(0);
    reinterpret_cast<T*>(I.phi[1])[o] = T(0);
}

// Temperature and liquid fraction (Eq. 8) of the current state into W1[0], W1[1].
template <typename T>
__global__ __launch_bounds__(PT_TX* PT_TY) void k_derived(const DevInst* __restrict__ insts,
                                                           const Tile* __restrict__ tiles)
{
    const Tile tile = tiles[blockIdx.x];
    const DevInst& I = insts[tile.inst];
    const int gx = tile.x0 + (int)threadIdx.x % PT_TX, gy = tile.y0 + (int)threadIdx.x / PT_TX;
    if (gx >= I.nx || gy >= I.ny) return;
    const size_t o = (size_t)gy * I.pitch + gx;
    T Tt, Fl;
    enthalpy_state<T>(coef<T>(I), reinterpret_cast<const T*>(I.W[0])[o], T(reinterpret_cast<const double*>(I.W[4])[o]),
                      Tt, Fl);
    reinterpret_cast<T*>(I.W1[0])[o] = Tt;
    reinterpret_cast<T*>(I.W1[1])[o] = Fl;
}

// Local heat flux Q = -lambda dT/dy on the south wall (Sec. 5.2, Fig. 15) of instance 0,
// one FP64 value per column into `out`: the second-order one-sided difference through
// the wall temperature and the first two cell centres, lambda of the wall cell (Eq. 11);
// zero unless the south wall holds a fixed temperature.
template <typename T>
__global__ __launch_bounds__(256) void k_wall_profile(const DevInst* __restrict__ insts, double* __restrict__ out)
{
    const DevInst& I = insts[0];
    const int i = blockIdx.x * 256 + (int)threadIdx.x;
    if (i >= I.nx) return;
    const Coef<T>& K = coef<T>(I);
    const GLOBAL T* He = gp<T>(I.W[0]);
    const GLOBAL double* C = gp<double>(I.W[4]);
    T T0, F0, T1, F1;
    enthalpy_state<T>(K, He[i], T(C[i]), T0, F0);
    enthalpy_state<T>(K, He[I.pitch + i], T(C[I.pitch + i]), T1, F1);
    const T ct = clamp01(T(C[i]));
    const double lam = double(mix3<T>(K.lam, ct * (T(1) - F0), ct));
    out[i] = I.heat_on ? -lam * (9.0 * double(T0) - double(T1) - 8.0 * I.tval[2]) / (3.0 * I.dx) : 0.0;
}

template <typename T>
hipError_t launch_wall_profile(const DevInst* insts, int nx, double* out, hipStream_t stream)
{
    if (nx <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_wall_profile<T>), dim3((nx + 255) / 256), dim3(256), 0, stream, insts, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init_fields(const DevInst* insts, const Tile* tiles, int ntiles, int kind,
                              double c_init, double t_init, double cx, double cy, double r,
                              hipStream_t stream)
{
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_init_fields<T>), dim3(ntiles), dim3(PT_TX * PT_TY), 0, stream, insts, tiles,
                       kind, c_init, t_init, cx, cy, r);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_derived(const DevInst* insts, const Tile* tiles, int ntiles, hipStream_t stream)
{
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_derived<T>), dim3(ntiles), dim3(PT_TX * PT_TY), 0, stream, insts, tiles);
    return hipGetLastError();
}


// ------------------------------------------------------------- multigrid

// Geometric multigrid for the compact magnetic system A u = f of one instance (not in
// the paper; the same fixed point as the sweeps, reached in fewer launches when the
// residual has to fall far). (A u)_c = sum over the cell's faces of w_f (u_c - u_nb),
// a wall face with its weight (2 mu_c at a fixed-potential wall, 0 at an insulating
// one) and u = 0 beyond it. Level 0 is the potential phi' itself with
// f = sum_f w_f (phi0_nb - phi0_c) (the constant term of the sweeps); a coarse level
// merges 2 x 2 cells (a last odd row or column maps to one cell), its face weight is
// the mean of the fine faces it covers, its right-hand side the sum of the children's
// residuals, and its correction is interpolated back to the children. Arrays: cells row-major
// with a pitch, x-face weights wx[j (nx+1) + i] (face i between cells i-1 and i),
// y-face weights wy[j nx + i] (face j between rows j-1 and j). One thread per cell or
// face; non-periodic domains.

// permeability of the level-0 cells (Eq. 2 with Eq. 11)
template <typename T>
__global__ __launch_bounds__(256) void k_mg_mu0(const DevInst* __restrict__ insts, T* __restrict__ mu)
{
    const DevInst& I = insts[0];
    const int c = blockIdx.x * 256 + (int)threadIdx.x;
    if (c >= I.nx * I.ny) return;
    const int i = c % I.nx, j = c / I.nx;
    const size_t o = (size_t)j * I.pitch + i;
    const Coef<T>& K = coef<T>(I);
    const T C = T(gp<double>(I.W[4])[o]);
    T Tt, Fl;
    enthalpy_state<T>(K, gp<T>(I.W[0])[o], C, Tt, Fl);
    mu[c] = mag_permeability<T>(K, clamp01(C), Fl);
}

// level-0 face weights from the permeability: the mean of two cells, 2 mu_c towards a
// fixed-potential wall, 0 at an insulating one
template <typename T>
__global__ __launch_bounds__(256) void k_mg_faces0(const DevInst* __restrict__ insts, const T* __restrict__ mu,
                                                   T* __restrict__ wx, T* __restrict__ wy)
{
    const DevInst& I = insts[0];
    const int nx = I.nx, ny = I.ny;
    const int nfx = (nx + 1) * ny, nfy = nx * (ny + 1);
    const int f = blockIdx.x * 256 + (int)threadIdx.x;
    if (f < nfx) {
        const int i = f % (nx + 1), j = f / (nx + 1);
        T w;
        if (i == 0) w = I.mbc[0] ? T(2) * mu[j * nx] : T(0);
        else if (i == nx) w = I.mbc[1] ? T(2) * mu[j * nx + nx - 1] : T(0);
        else w = T(0.5) * (mu[j * nx + i - 1] + mu[j * nx + i]);
        wx[f] = w;
    } else if (f < nfx + nfy) {
        const int g = f - nfx;
        const int i = g % nx, j = g / nx;
        T w;
        if (j == 0) w = I.mbc[2] ? T(2) * mu[i] : T(0);
        else if (j == ny) w = I.mbc[3] ? T(2) * mu[(ny - 1) * nx + i] : T(0);
        else w = T(0.5) * (mu[(j - 1) * nx + i] + mu[j * nx + i]);
        wy[g] = w;
    }
}

// level-0 right-hand side: the applied-field potential differences across each face
// (half of them across a wall face)
template <typename T>
__global__ __launch_bounds__(256) void k_mg_rhs0(const DevInst* __restrict__ insts, const T* __restrict__ wx,
                                                 const T* __restrict__ wy, T* __restrict__ f)
{
    const DevInst& I = insts[0];
    const int nx = I.nx, ny = I.ny;
    const int c = blockIdx.x * 256 + (int)threadIdx.x;
    if (c >= nx * ny) return;
    const int i = c % nx, j = c / nx;
    const Coef<T>& K = coef<T>(I);
    const T hx = K.h0x * K.dx, hy = K.h0y * K.dx;
    const T ww = wx[j * (nx + 1) + i], we = wx[j * (nx + 1) + i + 1];
    const T ws = wy[j * nx + i], wn = wy[(j + 1) * nx + i];
    f[c] = ww * (i == 0 ? T(0.5) * hx : hx) - we * (i == nx - 1 ? T(0.5) * hx : hx) +
           ws * (j == 0 ? T(0.5) * hy : hy) - wn * (j == ny - 1 ? T(0.5) * hy : hy);
}

// Cell widths along one axis of a multigrid level, in level-0 cells: every cell is w
// wide but the last, which is `last` wide (less when a halving had an odd count).
struct MgAxis {
    int n, w, last;
    __device__ __forceinline__ int width(int i) const { return i == n - 1 ? last : w; }
    __device__ __forceinline__ int start(int i) const { return i * w; }
    // distance between the centres of the cells on either side of face f (0..n), or from
    // the centre of a boundary cell to its wall
    __device__ __forceinline__ double face_dist(int f) const
    {
        return f == 0 ? 0.5 * width(0) : (f == n ? 0.5 * width(n - 1) : 0.5 * (width(f - 1) + width(f)));
    }
};

// coarse face weights: a face weight is the permeability times the face's length over
// the distance between the centres it connects (a two-dimensional conductance), so the
// coarse weight is the sum over the one or two fine faces it covers of weight x fine
// centre distance, over the coarse centre distance. For regular cells this is the mean
// of the fine faces; it also holds where a halving of an odd count leaves a narrower
// last cell.
template <typename T>
__global__ __launch_bounds__(256) void k_mg_coarsen(int nxf, int nyf, const T* __restrict__ wxf,
                                                    const T* __restrict__ wyf, int nxc, int nyc, T* __restrict__ wxc,
                                                    T* __restrict__ wyc, int wf, int lxf, int lyf, int lxc, int lyc)
{
    const MgAxis fx{nxf, wf, lxf}, fy{nyf, wf, lyf}, cx{nxc, 2 * wf, lxc}, cy{nyc, 2 * wf, lyc};
    const int nfx = (nxc + 1) * nyc, nfy = nxc * (nyc + 1);
    const int f = blockIdx.x * 256 + (int)threadIdx.x;
    if (f < nfx) {
        const int I = f % (nxc + 1), J = f / (nxc + 1);
        const int fi = min(2 * I, nxf);
        T sum = wxf[(2 * J) * (nxf + 1) + fi];
        if (2 * J + 1 < nyf) sum += wxf[(2 * J + 1) * (nxf + 1) + fi];
        wxc[f] = sum * T(fx.face_dist(fi) / cx.face_dist(I));
    } else if (f < nfx + nfy) {
        const int g = f - nfx;
        const int I = g % nxc, J = g / nxc;
        const int fj = min(2 * J, nyf);
        T sum = wyf[fj * nxf + 2 * I];
        if (2 * I + 1 < nxf) sum += wyf[fj * nxf + 2 * I + 1];
        wyc[g] = sum * T(fy.face_dist(fj) / cy.face_dist(J));
    }
}

// (A u)_c and the sum of the cell's face weights
template <typename T>
__device__ __forceinline__ void mg_apply(int nx, int ny, int pitch, const T* u, const T* wx, const T* wy, int i,
                                         int j, T& au, T& den, T& nbsum)
{
    const T ww = wx[j * (nx + 1) + i], we = wx[j * (nx + 1) + i + 1];
    const T ws = wy[j * nx + i], wn = wy[(j + 1) * nx + i];
    const T uw = i > 0 ? u[(size_t)j * pitch + i - 1] : T(0);
    const T ue = i < nx - 1 ? u[(size_t)j * pitch + i + 1] : T(0);
    const T us = j > 0 ? u[(size_t)(j - 1) * pitch + i] : T(0);
    const T un = j < ny - 1 ? u[(size_t)(j + 1) * pitch + i] : T(0);
    den = ww + we + ws + wn;
    nbsum = ww * uw + we * ue + ws * us + wn * un;
    au = den * u[(size_t)j * pitch + i] - nbsum;
}

// one red-black Gauss-Seidel colour pass, in place
template <typename T>
__global__ __launch_bounds__(256) void k_mg_smooth(int nx, int ny, int pitch, T* __restrict__ u,
                                                   const T* __restrict__ f, const T* __restrict__ wx,
                                                   const T* __restrict__ wy, int colour)
{
    // thread k takes the k-th cell of the colour in row-major order
    const int k = blockIdx.x * 256 + (int)threadIdx.x;
    const int half = (nx + 1) / 2;
    const int j = k / half;
    if (j >= ny) return;
    const int i = 2 * (k % half) + ((j + colour) & 1);
    if (i >= nx) return;
    T au, den, nbsum;
    mg_apply<T>(nx, ny, pitch, u, wx, wy, i, j, au, den, nbsum);
    if (den > T(0)) u[(size_t)j * pitch + i] = (f[j * nx + i] + nbsum) / den;
}

// coarse right-hand side (sum of the children's residuals) and a zero coarse correction
template <typename T>
__global__ __launch_bounds__(256) void k_mg_restrict(int nxf, int nyf, int pitchf, const T* __restrict__ uf,
                                                     const T* __restrict__ ff, const T* __restrict__ wxf,
                                                     const T* __restrict__ wyf, int nxc, int nyc, T* __restrict__ fc,
                                                     T* __restrict__ uc)
{
    const int c = blockIdx.x * 256 + (int)threadIdx.x;
    if (c >= nxc * nyc) return;
    const int I = c % nxc, J = c / nxc;
    T r = T(0);
    for (int b = 0; b < 2; b++)
        for (int a = 0; a < 2; a++) {
            const int i = 2 * I + a, j = 2 * J + b;
            if (i >= nxf || j >= nyf) continue;
            T au, den, nbsum;
            mg_apply<T>(nxf, nyf, pitchf, uf, wxf, wyf, i, j, au, den, nbsum);
            r += ff[j * nxf + i] - au;
        }
    fc[c] = r;
    uc[c] = T(0);
}

// the coarse cell a fine cell interpolates from besides its own, and that cell's weight,
// along one axis: linear in the cell-centre positions; beyond a wall the neighbour is the
// mirror image of the boundary cell (sign -1 at a fixed-potential wall)
struct MgInterp {
    int nb;
    double t, sign;
};
__device__ __forceinline__ MgInterp mg_interp(const MgAxis& f, const MgAxis& c, int i, int I, bool fixed_lo,
                                              bool fixed_hi)
{
    const double xf = f.start(i) + 0.5 * f.width(i);
    const double xc = c.start(I) + 0.5 * c.width(I);
    MgInterp r{I, 0.0, 1.0};
    if (xf == xc) return r;
    double xn;
    if (xf < xc) {
        if (I > 0) {
            r.nb = I - 1;
            xn = c.start(I - 1) + 0.5 * c.width(I - 1);
        } else {
            xn = -xc;   // mirror across the wall at 0
            r.sign = fixed_lo ? -1.0 : 1.0;
        }
    } else {
        if (I < c.n - 1) {
            r.nb = I + 1;
            xn = c.start(I + 1) + 0.5 * c.width(I + 1);
        } else {
            const double wall = c.start(I) + c.width(I);
            xn = 2.0 * wall - xc;
            r.sign = fixed_hi ? -1.0 : 1.0;
        }
    }
    r.t = (xf - xc) / (xn - xc);
    return r;
}

// add the coarse correction to every child, interpolated bilinearly from the four
// nearest coarse cell centres (for regular cells 9/16 its own, 3/16 each side
// neighbour, 1/16 the diagonal)
template <typename T>
__global__ __launch_bounds__(256) void k_mg_prolong(int nxf, int nyf, int pitchf, T* __restrict__ uf, int nxc,
                                                    int nyc, const T* __restrict__ uc, int fixed_walls, int wf,
                                                    int lxf, int lyf, int lxc, int lyc)
{
    const int c = blockIdx.x * 256 + (int)threadIdx.x;
    if (c >= nxf * nyf) return;
    const int i = c % nxf, j = c / nxf;
    const int I = i / 2, J = j / 2;
    const MgAxis fx{nxf, wf, lxf}, fy{nyf, wf, lyf}, cx{nxc, 2 * wf, lxc}, cy{nyc, 2 * wf, lyc};
    const MgInterp ax = mg_interp(fx, cx, i, I, fixed_walls & 1, (fixed_walls >> 1) & 1);
    const MgInterp ay = mg_interp(fy, cy, j, J, (fixed_walls >> 2) & 1, (fixed_walls >> 3) & 1);
    const T wx0 = T(1.0 - ax.t), wx1 = T(ax.t * ax.sign), wy0 = T(1.0 - ay.t), wy1 = T(ay.t * ay.sign);
    const T v = wy0 * (wx0 * uc[J * nxc + I] + wx1 * uc[J * nxc + ax.nb]) +
                wy1 * (wx0 * uc[ay.nb * nxc + I] + wx1 * uc[ay.nb * nxc + ax.nb]);
    uf[(size_t)j * pitchf + i] += v;
}

// the coarsest level (at most MG_COARSE x MG_COARSE cells) solved by red-black SOR in
// the LDS of one workgroup
template <typename T>
__global__ __launch_bounds__(1024) void k_mg_coarsest(int nx, int ny, int pitch, T* __restrict__ u,
                                                      const T* __restrict__ f, const T* __restrict__ wx,
                                                      const T* __restrict__ wy, int sweeps, double omega)
{
    constexpr int N = MG_COARSE * MG_COARSE;
    __shared__ T su[N];
    const int c = threadIdx.x;
    const bool mine = c < nx * ny;
    const int i = mine ? c % nx : 0, j = mine ? c / nx : 0;
    T ww = T(0), we = T(0), ws = T(0), wn = T(0), fc = T(0), rd = T(0);
    if (mine) {
        ww = wx[j * (nx + 1) + i];
        we = wx[j * (nx + 1) + i + 1];
        ws = wy[j * nx + i];
        wn = wy[(j + 1) * nx + i];
        fc = f[j * nx + i];
        const T den = ww + we + ws + wn;
        rd = den > T(0) ? T(1) / den : T(0);
        su[c] = u[(size_t)j * pitch + i];
    }
    __syncthreads();
    const T om = T(omega);
    for (int sw = 0; sw < 2 * sweeps; sw++) {
        if (mine && ((i + j) & 1) == (sw & 1) && rd > T(0)) {
            const T nb = (i > 0 ? ww * su[c - 1] : T(0)) + (i < nx - 1 ? we * su[c + 1] : T(0)) +
                         (j > 0 ? ws * su[c - nx] : T(0)) + (j < ny - 1 ? wn * su[c + nx] : T(0));
            su[c] = (T(1) - om) * su[c] + om * (fc + nb) * rd;
        }
        __syncthreads();
    }
    if (mine) u[(size_t)j * pitch + i] = su[c];
}

template <typename T>
hipError_t launch_mg_setup0(const DevInst* insts, int nx, int ny, T* mu_tmp, T* wx, T* wy, T* f, hipStream_t stream,
                            hipEvent_t e0)
{
    const int n = nx * ny, nf = (nx + 1) * ny + nx * (ny + 1);
    const hipError_t e = launch_timed(k_mg_mu0<T>, dim3((n + 255) / 256), dim3(256), stream, e0, nullptr, insts, mu_tmp);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_mg_faces0<T>), dim3((nf + 255) / 256), dim3(256), 0, stream, insts, mu_tmp, wx, wy);
    hipLaunchKernelGGL((k_mg_rhs0<T>), dim3((n + 255) / 256), dim3(256), 0, stream, insts, wx, wy, f);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mg_coarsen(int nxf, int nyf, const T* wxf, const T* wyf, int nxc, int nyc, T* wxc, T* wyc,
                             const int* geom, hipStream_t stream)
{
    const int nf = (nxc + 1) * nyc + nxc * (nyc + 1);
    hipLaunchKernelGGL((k_mg_coarsen<T>), dim3((nf + 255) / 256), dim3(256), 0, stream, nxf, nyf, wxf, wyf, nxc, nyc,
                       wxc, wyc, geom[0], geom[1], geom[2], geom[3], geom[4]);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mg_smooth(int nx, int ny, int pitch, T* u, const T* f, const T* wx, const T* wy, int sweeps,
                            hipStream_t stream)
{
    const int per_colour = ((nx + 1) / 2) * ny;
    for (int k = 0; k < 2 * sweeps; k++)
        hipLaunchKernelGGL((k_mg_smooth<T>), dim3((per_colour + 255) / 256), dim3(256), 0, stream, nx, ny, pitch, u,
                           f, wx, wy, k & 1);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mg_restrict(int nxf, int nyf, int pitchf, const T* uf, const T* ff, const T* wxf, const T* wyf,
                              int nxc, int nyc, T* fc, T* uc, hipStream_t stream)
{
    const int n = nxc * nyc;
    hipLaunchKernelGGL((k_mg_restrict<T>), dim3((n + 255) / 256), dim3(256), 0, stream, nxf, nyf, pitchf, uf, ff, wxf,
                       wyf, nxc, nyc, fc, uc);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mg_prolong(int nxf, int nyf, int pitchf, T* uf, int nxc, int nyc, const T* uc, int fixed_walls,
                             const int* geom, hipStream_t stream)
{
    const int n = nxf * nyf;
    hipLaunchKernelGGL((k_mg_prolong<T>), dim3((n + 255) / 256), dim3(256), 0, stream, nxf, nyf, pitchf, uf, nxc, nyc,
                       uc, fixed_walls, geom[0], geom[1], geom[2], geom[3], geom[4]);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_mg_coarsest(int nx, int ny, int pitch, T* u, const T* f, const T* wx, const T* wy, int sweeps,
                              double omega, hipStream_t stream)
{
    if (nx * ny > MG_COARSE * MG_COARSE) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_mg_coarsest<T>), dim3(1), dim3(1024), 0, stream, nx, ny, pitch, u, f, wx, wy, sweeps, omega);
    return hipGetLastError();
}

#define LBFS_INSTANTIATE(T)                                                                          \
    template hipError_t launch_stage<T>(int, int, int, const DevInst*, const Tile*, int, hipStream_t, hipEvent_t, \
                                        hipEvent_t);                                                   \
    template hipError_t launch_stage_fused<T>(int, int, int, double, const DevInst*, const Tile*, int, hipStream_t, \
                                              hipEvent_t, hipEvent_t);                                 \
    template hipError_t launch_mag<T>(int, int, double, int, int, int*, const DevInst*, const Tile*, int, hipStream_t, \
                                      hipEvent_t, hipEvent_t, int);                                    \
    template hipError_t launch_mag_lbfs<T>(int, int, int, int*, const DevInst*, const Tile*, int, hipStream_t, \
                                           hipEvent_t, hipEvent_t, int);                               \
    template hipError_t launch_state_partials<T>(int, const DevInst*, const Tile*, int, hipStream_t); \
    template hipError_t launch_init_fields<T>(const DevInst*, const Tile*, int, int, double, double, \
                                              double, double, double, hipStream_t);                 \
    template hipError_t launch_derived<T>(const DevInst*, const Tile*, int, hipStream_t);                 \
    template hipError_t launch_wall_profile<T>(const DevInst*, int, double*, hipStream_t);                \
    template hipError_t launch_mg_setup0<T>(const DevInst*, int, int, T*, T*, T*, T*, hipStream_t, hipEvent_t); \
    template hipError_t launch_mg_coarsen<T>(int, int, const T*, const T*, int, int, T*, T*, const int*,     \
                                             hipStream_t);                                                \
    template hipError_t launch_mg_smooth<T>(int, int, int, T*, const T*, const T*, const T*, int, hipStream_t); \
    template hipError_t launch_mg_restrict<T>(int, int, int, const T*, const T*, const T*, const T*, int, int, T*, T*, \
                                              hipStream_t);                                            \
    template hipError_t launch_mg_prolong<T>(int, int, int, T*, int, int, const T*, int, const int*,     \
                                             hipStream_t);                                                \
    template hipError_t launch_mg_coarsest<T>(int, int, int, T*, const T*, const T*, const T*, int, double, \
                                              hipStream_t);

LBFS_INSTANTIATE(float)
LBFS_INSTANTIATE(double)

}  // namespace lbfs

/*
 * lbfs_oracle.c -- plain FP64 CPU oracle of the enthalpy-based LBFS (arXiv 2511.10257).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark load this file's library; the HIP product never does. It is written
 * to be checked against the paper by eye: every face flux is evaluated literally as the
 * moments of the nine star distributions, with no algebraic shortcut, no blocking and
 * no fusion. Single threaded, FP64 throughout.
 *
 * Method, in the paper's order (Table 1, "computational procedure"):
 *   magnetic potential  : Eq. 4, discretised by the magnetic LBFS flux of Sec. 3.1 at
 *                         delta_t = dx/2 (a compact 5-point system) and relaxed by
 *                         red-black Gauss-Seidel/SOR sweeps, or (mag_method 1) the
 *                         LBFS pseudo-time solve itself: m* fluxes built literally
 *                         (Eqs. 13, 16, 18, 44, 45) and Eq. 17 advanced by SSP-RK3;
 *   Kelvin force        : Eq. 6, last line;
 *   thermal/flow/phase  : Eq. 38-46 (cell-centred FVM, Eq. 44 reconstruction, Eq. 45
 *                         compatibility, star distributions Eqs. 16, 22, 32, 33,
 *                         fluxes Eq. 43, sources Eq. 41), advanced by third-order
 *                         strong-stability-preserving Runge-Kutta;
 *   phase change        : Eq. 8 after the Runge-Kutta step.
 * Where the paper is garbled or silent the readings below are used (each is listed in
 * the design notes of the repository):
 *   - D2Q9 weights 4/9, 1/9, 1/36; diagonal velocities (1,1), (-1,1), (-1,-1), (1,-1).
 *   - delta_t (streaming step) is a parameter; the product fixes it to dx/2.
 *   - Eq. 44 points with e_a.n = 0 take the average of both one-sided reconstructions.
 *   - Face density and face chemical potential are the reconstructions at the face
 *     centre (the a = 0 point); face mu, lambda, Cp are two-cell arithmetic means.
 *   - Eq. 32 is used with the sign of Eqs. 16, 22, 33 (f* = f_eq + (1 - 1/2tau) f_neq),
 *     the sign that makes the stress viscous.
 *   - mu_c = 2 beta C (C-1)(2C-1) - kappa lap(C) (the sign for which the tanh profile
 *     of width xi is an equilibrium).
 *   - Eq. 8 with Ts = Tl = Tm, local latent heat Ct*L, branch heat capacities of the
 *     solid-gas and liquid-gas mixtures; Fs = Ct (1 - Fl); Eq. 11 with Ct = clamp(C).
 *   - dFs/dt is lagged by one step; F_IBM = -rho u Fs / Dt (direct forcing).
 *   - Walls: zero mass and order-parameter flux; fixed-temperature walls conduct
 *     through the half cell; momentum flux from the same LBFS face formula with
 *     mirrored ghost cells (no-slip). A wall with a contact angle other than 90 degrees
 *     gives the order parameter's ghost cells the wall-normal gradient of that angle
 *     (wetting; the paper does not give its condition).
 *   - Magnetic LBFS: the flux sum_a e_a m*_a that Eqs. 15-16 give is -D mu grad(phi),
 *     so Eq. 17 is a diffusion towards Eq. 4 (Eq. 18 prints the opposite sign);
 *     tau_m uses the mean permeability of the face's two cells; the pseudo-time step
 *     is a parameter, by default the stable dx^2 / (4 D mu_max); the initial solve
 *     uses the sweeps whatever the per-step method (same fixed point).
 */
#include "lbfs_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define G 3          /* ghost layers */
#define NREC 8       /* variables reconstructed at the Eq. 44 points */
enum { R_P, R_U, R_V, R_RHO, R_C, R_MUC, R_T, R_HE };

/* D2Q9, Eq. 14 and Fig. 1 */
static const double EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const double EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WA[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0;

enum { K_EVEN, K_ODD, K_TEMP, K_WET };

struct orc_sim {
    orc_params p;
    int nx, ny, px, py;
    double cpref, beta, kappa, qg;
    double t, step, vol0, res;
    double *W[5], *Wa[5], *Wb[5], *R[5];
    double *phi, *S, *mum, *fmg[2];
    /* per-evaluation work arrays (padded) */
    double *val[NREC], *gx[NREC], *gy[NREC];
    double *mu, *lam, *cp, *fs;
    double *fx[5], *fy[5];
    /* magnetic LBFS pseudo-time solve: RK3 stage values, rate, cell gradients, fluxes */
    double *mph[2], *mL, *mgx, *mgy, *mfx, *mfy;
};

#define IX(s, i, j) (((j) + G) * (s)->px + ((i) + G))

static double clamp01(double c) { return c < 0.0 ? 0.0 : (c > 1.0 ? 1.0 : c); }

/* Eq. 11: property of the solid / liquid / gas mixture */
static double mix3(const double g[3], double fs, double ct)
{
    return fs * g[0] + (1.0 - fs) * ct * g[1] + (1.0 - fs) * (1.0 - ct) * g[2];
}

void orc_lattice(double* ex, double* ey, double* w)
{
    for (int a = 0; a < 9; a++) { ex[a] = EX[a]; ey[a] = EY[a]; w[a] = WA[a]; }
}

/* Eq. 8: liquid fraction and temperature from the total enthalpy. */
void orc_enthalpy_state(const orc_params* p, double He, double C, double* T, double* Fl)
{
    double ct = clamp01(C);
    double cp_sol = ct * p->cp[0] + (1.0 - ct) * p->cp[2];
    double cp_liq = ct * p->cp[1] + (1.0 - ct) * p->cp[2];
    double Ts = p->t_melt, Tl = p->t_liquidus;
    double Hes = cp_sol * Ts;                    /* H_es = Cp,s Ts      */
    double Hel = cp_liq * Tl + ct * p->latent;   /* H_el = Cp,l Tl + L  */
    if (He > Hel) {
        *Fl = 1.0;
        *T = Tl + (He - Hel) / cp_liq;
    } else if (He >= Hes && Hel > Hes) {
        *Fl = (He - Hes) / (Hel - Hes);
        *T = Ts + *Fl * (Tl - Ts);
    } else {
        *Fl = 0.0;
        *T = He / cp_sol;
    }
}

/* Eq. 28 (and f^{eq-m} of Sec. 3.3 when rho is the face density) */
static double f_eq(int a, double pr, double rho, double u, double v)
{
    double eu = EX[a] * u + EY[a] * v, uu = u * u + v * v;
    return WA[a] * (pr + rho * CS2 * (eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2)));
}

/* Eq. 29 */
static double g_eq(const struct orc_sim* s, int a, double C, double muc, double u, double v)
{
    if (a == 0) return C - muc * s->qg * (1.0 - WA[0]) / CS2;
    return WA[a] * (muc * s->qg + C * (EX[a] * u + EY[a] * v)) / CS2;
}

/* Eq. 20 */
static double h_eq(double cpref, int a, double He, double T, double cp, double u, double v)
{
    double uu = u * u + v * v;
    if (a == 0) return He - cpref * T + WA[0] * cp * T * (cpref / cp - uu / (2.0 * CS2));
    double eu = EX[a] * u + EY[a] * v;
    return WA[a] * cp * T * (cpref / cp + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
}

void orc_equilibria(const orc_params* p, double pr, double rho, double u, double v,
                    double C, double muc, double He, double T, double cp,
                    double* feq, double* geq, double* heq)
{
    struct orc_sim tmp;
    memset(&tmp, 0, sizeof tmp);
    tmp.p = *p;
    tmp.qg = p->mobility / ((p->tau_g - 0.5) * p->dt_stream);
    double cpref = 0.5 * (p->cp[0] + p->cp[1]);
    for (int a = 0; a < 9; a++) {
        feq[a] = f_eq(a, pr, rho, u, v);
        geq[a] = g_eq(&tmp, a, C, muc, u, v);
        heq[a] = h_eq(cpref, a, He, T, cp, u, v);
    }
}

void orc_params_from_dimless(orc_params* p, double ste, double t_wall, double bo_m)
{
    p->latent = p->cp[1] * (p->t_melt - t_wall) / ste;
    p->h0 = sqrt(bo_m * p->sigma / (p->mu0 * 2.0 * p->drop_r));
}

static double* zalloc(size_t n) { return (double*)calloc(n, sizeof(double)); }

orc_sim* orc_new(const orc_params* pin)
{
    const orc_params* p = pin;
    if (p->nx < 4 || p->ny < 4 || p->dx <= 0 || p->dt < 0 || p->dt_stream <= 0) return NULL;
    if (p->tau_g <= 0.5 || p->xi <= 0) return NULL;
    if (!(p->t_liquidus >= p->t_melt)) return NULL;
    if (p->mag_method < 0 || p->mag_method > 1) return NULL;
    if (p->mag_method == 1 && !(p->mag_lbfs_d > 0.0)) return NULL;
    if (p->mag_max_iters < 0 || (p->mag_max_iters > 0 && (p->sweeps <= 0 || !(p->mag_tol >= 0.0)))) return NULL;
    for (int w = 0; w < 4; w++)
        if (!(p->contact_angle[w] > 0.0 && p->contact_angle[w] < 180.0)) return NULL;
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    s->p = *p;
    if (s->p.dt == 0.0) {
        /* automatic step: dx/2 unless the largest kinematic viscosity or thermal
           diffusivity D needs 0.4 dx^2 / D */
        double D = 0.0;
        for (int k = 0; k < 3; k++) {
            double nu = p->mu[k] / p->rho[k], al = p->lam[k] / (p->rho[k] * p->cp[k]);
            if (nu > D) D = nu;
            if (al > D) D = al;
        }
        double diff = D > 0.0 ? 0.4 * p->dx * p->dx / D : 0.5 * p->dx;
        s->p.dt = 0.5 * p->dx < diff ? 0.5 * p->dx : diff;
    }
    s->nx = p->nx; s->ny = p->ny;
    s->px = p->nx + 2 * G; s->py = p->ny + 2 * G;
    s->cpref = 0.5 * (p->cp[0] + p->cp[1]);        /* Sec. 3.2 */
    s->beta = 12.0 * p->sigma / p->xi;             /* Sec. 2 */
    s->kappa = 1.5 * p->xi * p->sigma;
    s->qg = p->mobility / ((p->tau_g - 0.5) * p->dt_stream);   /* M_c = (tau_g - 1/2) Q_g delta_t */
    size_t n = (size_t)s->px * s->py;
    for (int k = 0; k < 5; k++) {
        s->W[k] = zalloc(n); s->Wa[k] = zalloc(n); s->Wb[k] = zalloc(n); s->R[k] = zalloc(n);
        s->fx[k] = zalloc((size_t)(p->nx + 1) * p->ny);
        s->fy[k] = zalloc((size_t)p->nx * (p->ny + 1));
    }
    s->phi = zalloc(n); s->S = zalloc(n); s->mum = zalloc(n);
    s->fmg[0] = zalloc(n); s->fmg[1] = zalloc(n);
    for (int k = 0; k < NREC; k++) { s->val[k] = zalloc(n); s->gx[k] = zalloc(n); s->gy[k] = zalloc(n); }
    s->mu = zalloc(n); s->lam = zalloc(n); s->cp = zalloc(n); s->fs = zalloc(n);
    s->mph[0] = zalloc(n); s->mph[1] = zalloc(n); s->mL = zalloc(n); s->mgx = zalloc(n); s->mgy = zalloc(n);
    s->mfx = zalloc((size_t)(p->nx + 1) * p->ny); s->mfy = zalloc((size_t)p->nx * (p->ny + 1));
    return s;
}

void orc_free(orc_sim* s)
{
    if (!s) return;
    for (int k = 0; k < 5; k++) { free(s->W[k]); free(s->Wa[k]); free(s->Wb[k]); free(s->R[k]); free(s->fx[k]); free(s->fy[k]); }
    free(s->phi); free(s->S); free(s->mum); free(s->fmg[0]); free(s->fmg[1]);
    for (int k = 0; k < NREC; k++) { free(s->val[k]); free(s->gx[k]); free(s->gy[k]); }
    free(s->mu); free(s->lam); free(s->cp); free(s->fs);
    free(s->mph[0]); free(s->mph[1]); free(s->mL); free(s->mgx); free(s->mgy); free(s->mfx); free(s->mfy);
    free(s);
}

/* ------------------------------------------------------------------ ghosts */

/* value of a ghost cell mirroring interior value v across wall w */
/* value of the ghost cell k layers beyond wall w (k = 0 nearest) that mirrors interior
   value v; K_WET (the order parameter) adds the wall-normal gradient of the contact
   angle: n.grad C = -(4/xi) cos(theta) C (1 - C) (n into the fluid, the equilibrium
   tanh profile's |grad C| = (4/xi) C (1 - C)), over the 2k+1 cells between ghost and
   mirror cell, with C of the mirror cell */
static double reflect(const orc_sim* s, double v, int kind, int w, int k)
{
    if (kind == K_ODD) return -v;
    if (kind == K_TEMP && s->p.tbc[w] == 1) return 2.0 * s->p.tval[w] - v;
    if (kind == K_WET && s->p.contact_angle[w] != 90.0) {
        double c = clamp01(v);
        double g = 4.0 / s->p.xi * cos(s->p.contact_angle[w] * M_PI / 180.0) * c * (1.0 - c);
        return v + (2 * k + 1) * s->p.dx * g;
    }
    return v;
}

/* Fill G ghost layers: x direction on the interior rows first, then y direction on all
   columns (so a corner ghost is the y-mirror of the x-mirror). */
static void fill_ghosts(const orc_sim* s, double* a, int kind)
{
    int nx = s->nx, ny = s->ny;
    for (int j = 0; j < ny; j++)
        for (int k = 0; k < G; k++) {
            if (s->p.periodic[0]) {
                a[IX(s, -1 - k, j)] = a[IX(s, nx - 1 - k, j)];
                a[IX(s, nx + k, j)] = a[IX(s, k, j)];
            } else {
                a[IX(s, -1 - k, j)] = reflect(s, a[IX(s, k, j)], kind, 0, k);
                a[IX(s, nx + k, j)] = reflect(s, a[IX(s, nx - 1 - k, j)], kind, 1, k);
            }
        }
    for (int i = -G; i < nx + G; i++)
        for (int k = 0; k < G; k++) {
            if (s->p.periodic[1]) {
                a[IX(s, i, -1 - k)] = a[IX(s, i, ny - 1 - k)];
                a[IX(s, i, ny + k)] = a[IX(s, i, k)];
            } else {
                a[IX(s, i, -1 - k)] = reflect(s, a[IX(s, i, k)], kind, 2, k);
                a[IX(s, i, ny + k)] = reflect(s, a[IX(s, i, ny - 1 - k)], kind, 3, k);
            }
        }
}

/* ------------------------------------------------------------- magnetics */

static double phi_applied(const orc_sim* s, double x, double y)
{
    double th = s->p.angle_deg * M_PI / 180.0;
    return -s->p.h0 * (x * cos(th) + y * sin(th));   /* H = -grad(phi) = H0 (cos, sin) */
}

/* mu_m = mu0 (1 + chi) (Eq. 2), chi by Eq. 11 from the current C and He */
static void compute_mum(orc_sim* s)
{
    for (int j = 0; j < s->ny; j++)
        for (int i = 0; i < s->nx; i++) {
            int c = IX(s, i, j);
            double T, Fl, ct = clamp01(s->W[ORC_C][c]);
            orc_enthalpy_state(&s->p, s->W[ORC_HE][c], s->W[ORC_C][c], &T, &Fl);
            double fs = ct * (1.0 - Fl);
            s->mum[c] = s->p.mu0 * (1.0 + mix3(s->p.chi, fs, ct));
        }
}

/* Sum over the four faces of cell (i,j) of w_f * phi_nb and w_f, where w_f is the face
   permeability of the compact magnetic flux (mean of the two cells; 2 mu_i towards a
   fixed-potential wall at half-cell distance; no term at an insulating wall). */
static void mag_faces(const orc_sim* s, int i, int j, double* num, double* den)
{
    static const int DI[4] = {-1, 1, 0, 0}, DJ[4] = {0, 0, -1, 1};
    int c = IX(s, i, j);
    double dx = s->p.dx;
    *num = 0.0; *den = 0.0;
    for (int d = 0; d < 4; d++) {
        int ii = i + DI[d], jj = j + DJ[d];
        int axis = d < 2 ? 0 : 1;
        int inside = ii >= 0 && ii < s->nx && jj >= 0 && jj < s->ny;
        if (!inside && s->p.periodic[axis]) {
            ii = (ii + s->nx) % s->nx; jj = (jj + s->ny) % s->ny; inside = 1;
        }
        if (inside) {
            int nb = IX(s, ii, jj);
            double w = 0.5 * (s->mum[c] + s->mum[nb]);
            *num += w * s->phi[nb]; *den += w;
        } else if (s->p.mbc[d] == 1) {
            double xw = (i + 0.5) * dx + 0.5 * dx * DI[d];
            double yw = (j + 0.5) * dx + 0.5 * dx * DJ[d];
            double w = 2.0 * s->mum[c];
            *num += w * phi_applied(s, xw, yw); *den += w;
        }
    }
}

static void rb_pass(orc_sim* s, int color, double omega)
{
    for (int j = 0; j < s->ny; j++)
        for (int i = 0; i < s->nx; i++) {
            if (((i + j) & 1) != color) continue;
            double num, den;
            mag_faces(s, i, j, &num, &den);
            int c = IX(s, i, j);
            if (den > 0.0) s->phi[c] = (1.0 - omega) * s->phi[c] + omega * num / den;
        }
}

double orc_mag_residual(orc_sim* s)
{
    double r2 = 0.0;
    for (int j = 0; j < s->ny; j++)
        for (int i = 0; i < s->nx; i++) {
            double num, den;
            mag_faces(s, i, j, &num, &den);
            double r = num - den * s->phi[IX(s, i, j)];
            r2 += r * r;
        }
    return sqrt(r2);
}

double orc_mag_sweeps(orc_sim* s, int nsweeps, double omega)
{
    compute_mum(s);
    for (int k = 0; k < nsweeps; k++) { rb_pass(s, 0, omega); rb_pass(s, 1, omega); }
    return orc_mag_residual(s);
}

/* ------------------------------------------------ magnetic LBFS (Sec. 3.1) */

/* Ghost layers of a potential for the LBFS construction: a fixed-potential wall keeps
   the applied potential at the wall (odd reflection about it), an insulating wall
   mirrors the potential (zero normal derivative), a periodic axis wraps. The x
   direction on the interior rows first, then y on all columns. */
static void fill_phi_ghosts(const orc_sim* s, double* a)
{
    int nx = s->nx, ny = s->ny;
    double dx = s->p.dx;
    for (int j = 0; j < ny; j++) {
        double y = (j + 0.5) * dx;
        for (int k = 0; k < G; k++) {
            if (s->p.periodic[0]) {
                a[IX(s, -1 - k, j)] = a[IX(s, nx - 1 - k, j)];
                a[IX(s, nx + k, j)] = a[IX(s, k, j)];
            } else {
                double vw = a[IX(s, k, j)], ve = a[IX(s, nx - 1 - k, j)];
                a[IX(s, -1 - k, j)] = s->p.mbc[0] == 1 ? 2.0 * phi_applied(s, 0.0, y) - vw : vw;
                a[IX(s, nx + k, j)] = s->p.mbc[1] == 1 ? 2.0 * phi_applied(s, nx * dx, y) - ve : ve;
            }
        }
    }
    for (int i = -G; i < nx + G; i++) {
        double x = (i + 0.5) * dx;
        for (int k = 0; k < G; k++) {
            if (s->p.periodic[1]) {
                a[IX(s, i, -1 - k)] = a[IX(s, i, ny - 1 - k)];
                a[IX(s, i, ny + k)] = a[IX(s, i, k)];
            } else {
                double vs = a[IX(s, i, k)], vn = a[IX(s, i, ny - 1 - k)];
                a[IX(s, i, -1 - k)] = s->p.mbc[2] == 1 ? 2.0 * phi_applied(s, x, 0.0) - vs : vs;
                a[IX(s, i, ny + k)] = s->p.mbc[3] == 1 ? 2.0 * phi_applied(s, x, ny * dx) - vn : vn;
            }
        }
    }
}

/* Normal flux sum_a e_a.n m*_a (Eq. 18) through the face between cell (iL, jL) and its
   neighbour along `axis`. The potential at the nine points x_f - e_a delta_t comes
   from Eq. 44 (the cell on the point's side and its gradient; the two one-sided values
   averaged for points on the face line), the face potential from the compatibility
   sum of Eq. 45, the equilibria at the face and at the points from Eq. 13, the
   non-equilibrium part and m* from Eq. 16 with tau_m = 1/2 + mu_f D / (cs^2 delta_t),
   mu_f the mean permeability of the two cells. */
static double lbfs_mag_face(const orc_sim* s, const double* ph, int axis, int iL, int jL, double D)
{
    double dx = s->p.dx, dts = s->p.dt_stream;
    int iR = iL + (axis == 0), jR = jL + (axis == 1);
    int cL = IX(s, iL, jL), cR = IX(s, iR, jR);
    double xL = (iL + 0.5) * dx, yL = (jL + 0.5) * dx, xR = (iR + 0.5) * dx, yR = (jR + 0.5) * dx;
    double xf = 0.5 * (xL + xR), yf = 0.5 * (yL + yR);
    double pv[9], phif = 0.0;
    for (int a = 0; a < 9; a++) {
        double px = xf - EX[a] * dts, py = yf - EY[a] * dts;
        double en = axis == 0 ? EX[a] : EY[a];
        double vL = ph[cL] + (px - xL) * s->mgx[cL] + (py - yL) * s->mgy[cL];
        double vR = ph[cR] + (px - xR) * s->mgx[cR] + (py - yR) * s->mgy[cR];
        pv[a] = en > 0.0 ? vL : (en < 0.0 ? vR : 0.5 * (vL + vR));
        phif += WA[a] * pv[a];
    }
    double muf = 0.5 * (s->mum[cL] + s->mum[cR]);
    double taum = 0.5 + muf * D / (CS2 * dts);
    double F = 0.0;
    for (int a = 0; a < 9; a++) {
        double en = axis == 0 ? EX[a] : EY[a];
        double meq_f = WA[a] * phif;
        double meq_p = WA[a] * pv[a];
        double mneq = -taum * (meq_f - meq_p);
        double mstar = meq_f + (1.0 - 0.5 / taum) * mneq;
        F += en * mstar;
    }
    return F;
}

/* all face fluxes of potential ph into s->mfx / s->mfy (permeability and its ghosts
   already in s->mum) */
static void lbfs_mag_fluxes(orc_sim* s, double* ph, double D)
{
    int nx = s->nx, ny = s->ny;
    double dx = s->p.dx;
    fill_phi_ghosts(s, ph);
    for (int j = -G + 1; j < ny + G - 1; j++)
        for (int i = -G + 1; i < nx + G - 1; i++) {
            int c = IX(s, i, j);
            s->mgx[c] = (ph[IX(s, i + 1, j)] - ph[IX(s, i - 1, j)]) / (2.0 * dx);
            s->mgy[c] = (ph[IX(s, i, j + 1)] - ph[IX(s, i, j - 1)]) / (2.0 * dx);
        }
    for (int j = 0; j < ny; j++)
        for (int i = 0; i <= nx; i++) s->mfx[j * (nx + 1) + i] = lbfs_mag_face(s, ph, 0, i - 1, j, D);
    for (int j = 0; j <= ny; j++)
        for (int i = 0; i < nx; i++) s->mfy[j * nx + i] = lbfs_mag_face(s, ph, 1, i, j - 1, D);
}

/* d(phi)/d(tau) of Eq. 17 by the finite-volume balance of Eq. 42 */
static void lbfs_mag_rate(orc_sim* s, double* ph, double D, double* L)
{
    int nx = s->nx, ny = s->ny;
    double dx = s->p.dx;
    lbfs_mag_fluxes(s, ph, D);
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++)
            L[IX(s, i, j)] = -(s->mfx[j * (nx + 1) + i + 1] - s->mfx[j * (nx + 1) + i] +
                               s->mfy[(j + 1) * nx + i] - s->mfy[j * nx + i]) / dx;
}

static void mag_permeability_with_ghosts(orc_sim* s)
{
    compute_mum(s);
    fill_ghosts(s, s->mum, K_EVEN);
}

double orc_mag_lbfs_dtau(const orc_params* p, double D)
{
    /* Every row of the discrete operator sums in absolute value to at most
       8 D mu_max / dx^2 and SSP-RK3 is stable on the negative real axis up to about
       -2.51, so this step (|z| <= 2) keeps every mode stable. The mixture permeability
       (Eq. 11) never exceeds that of the most permeable phase. */
    double m = 1.0 + p->chi[0];
    for (int k = 1; k < 3; k++)
        if (1.0 + p->chi[k] > m) m = 1.0 + p->chi[k];
    return p->dx * p->dx / (4.0 * D * p->mu0 * m);
}

double orc_mag_lbfs(orc_sim* s, int nsteps, double D, double dtau)
{
    int nx = s->nx, ny = s->ny;
    if (dtau <= 0.0) dtau = orc_mag_lbfs_dtau(&s->p, D);
    mag_permeability_with_ghosts(s);
    double *u0 = s->phi, *u1 = s->mph[0], *u2 = s->mph[1], *L = s->mL;
    for (int n = 0; n < nsteps; n++) {
        lbfs_mag_rate(s, u0, D, L);
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                int c = IX(s, i, j);
                u1[c] = u0[c] + dtau * L[c];
            }
        lbfs_mag_rate(s, u1, D, L);
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                int c = IX(s, i, j);
                u2[c] = 0.75 * u0[c] + 0.25 * (u1[c] + dtau * L[c]);
            }
        lbfs_mag_rate(s, u2, D, L);
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                int c = IX(s, i, j);
                u0[c] = u0[c] / 3.0 + 2.0 / 3.0 * (u2[c] + dtau * L[c]);
            }
    }
    return orc_mag_residual(s);
}

void orc_mag_lbfs_fluxes(orc_sim* s, double D, double* fx, double* fy)
{
    int nx = s->nx, ny = s->ny;
    mag_permeability_with_ghosts(s);
    lbfs_mag_fluxes(s, s->phi, D);
    memcpy(fx, s->mfx, (size_t)(nx + 1) * ny * sizeof(double));
    memcpy(fy, s->mfy, (size_t)nx * (ny + 1) * sizeof(double));
}

/* Kelvin force (Eq. 6): H = -grad(phi) and F = (mu0 chi / 2) grad|H|^2, central
   differences; ghost phi by the wall condition, ghost |H|^2 mirrored. */
static void kelvin(orc_sim* s)
{
    int nx = s->nx, ny = s->ny;
    double dx = s->p.dx;
    double* ph = s->Wa[0];   /* scratch */
    double* h2 = s->Wa[1];
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) ph[IX(s, i, j)] = s->phi[IX(s, i, j)];
    for (int j = 0; j < ny; j++) {
        if (s->p.periodic[0]) {
            ph[IX(s, -1, j)] = ph[IX(s, nx - 1, j)]; ph[IX(s, nx, j)] = ph[IX(s, 0, j)];
        } else {
            double y = (j + 0.5) * dx;
            ph[IX(s, -1, j)] = s->p.mbc[0] == 1 ? 2.0 * phi_applied(s, 0.0, y) - ph[IX(s, 0, j)] : ph[IX(s, 0, j)];
            ph[IX(s, nx, j)] = s->p.mbc[1] == 1 ? 2.0 * phi_applied(s, nx * dx, y) - ph[IX(s, nx - 1, j)] : ph[IX(s, nx - 1, j)];
        }
    }
    for (int i = 0; i < nx; i++) {
        if (s->p.periodic[1]) {
            ph[IX(s, i, -1)] = ph[IX(s, i, ny - 1)]; ph[IX(s, i, ny)] = ph[IX(s, i, 0)];
        } else {
            double x = (i + 0.5) * dx;
            ph[IX(s, i, -1)] = s->p.mbc[2] == 1 ? 2.0 * phi_applied(s, x, 0.0) - ph[IX(s, i, 0)] : ph[IX(s, i, 0)];
            ph[IX(s, i, ny)] = s->p.mbc[3] == 1 ? 2.0 * phi_applied(s, x, ny * dx) - ph[IX(s, i, ny - 1)] : ph[IX(s, i, ny - 1)];
        }
    }
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            double hx = -(ph[IX(s, i + 1, j)] - ph[IX(s, i - 1, j)]) / (2.0 * dx);
            double hy = -(ph[IX(s, i, j + 1)] - ph[IX(s, i, j - 1)]) / (2.0 * dx);
            h2[IX(s, i, j)] = hx * hx + hy * hy;
        }
    fill_ghosts(s, h2, K_EVEN);
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            int c = IX(s, i, j);
            double T, Fl, ct = clamp01(s->W[ORC_C][c]);
            orc_enthalpy_state(&s->p, s->W[ORC_HE][c], s->W[ORC_C][c], &T, &Fl);
            double chi = mix3(s->p.chi, ct * (1.0 - Fl), ct);
            double k = 0.5 * s->p.mu0 * chi;
            s->fmg[0][c] = k * (h2[IX(s, i + 1, j)] - h2[IX(s, i - 1, j)]) / (2.0 * dx);
            s->fmg[1][c] = k * (h2[IX(s, i, j + 1)] - h2[IX(s, i, j - 1)]) / (2.0 * dx);
        }
}

/* ---------------------------------------------------- cell-derived fields */

static void primitives(orc_sim* s, double* const Win[5])
{
    int nx = s->nx, ny = s->ny;
    double dx = s->p.dx;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            int c = IX(s, i, j);
            double He = Win[ORC_HE][c], C = Win[ORC_C][c];
            double T, Fl, ct = clamp01(C);
            orc_enthalpy_state(&s->p, He, C, &T, &Fl);
            double fs = ct * (1.0 - Fl);
            double rho = mix3(s->p.rho, fs, ct);
            s->val[R_P][c] = Win[ORC_P][c];
            s->val[R_U][c] = Win[ORC_MX][c] / (rho * CS2);
            s->val[R_V][c] = Win[ORC_MY][c] / (rho * CS2);
            s->val[R_RHO][c] = rho;
            s->val[R_C][c] = C;
            s->val[R_T][c] = T;
            s->val[R_HE][c] = He;
            s->mu[c] = mix3(s->p.mu, fs, ct);
            s->lam[c] = mix3(s->p.lam, fs, ct);
            s->cp[c] = mix3(s->p.cp, fs, ct);
            s->fs[c] = fs;
        }
    fill_ghosts(s, s->val[R_P], K_EVEN);
    fill_ghosts(s, s->val[R_U], K_ODD);
    fill_ghosts(s, s->val[R_V], K_ODD);
    fill_ghosts(s, s->val[R_RHO], K_EVEN);
    fill_ghosts(s, s->val[R_C], K_WET);
    fill_ghosts(s, s->val[R_T], K_TEMP);
    fill_ghosts(s, s->val[R_HE], K_EVEN);
    fill_ghosts(s, s->mu, K_EVEN);
    fill_ghosts(s, s->lam, K_EVEN);
    fill_ghosts(s, s->cp, K_EVEN);
    /* chemical potential (Sec. 2, sign per the equilibrium reading), 5-point Laplacian */
    double* C = s->val[R_C];
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            int c = IX(s, i, j);
            double lap = (C[IX(s, i + 1, j)] + C[IX(s, i - 1, j)] + C[IX(s, i, j + 1)] +
                          C[IX(s, i, j - 1)] - 4.0 * C[c]) / (dx * dx);
            s->val[R_MUC][c] = 2.0 * s->beta * C[c] * (C[c] - 1.0) * (2.0 * C[c] - 1.0) - s->kappa * lap;
        }
    fill_ghosts(s, s->val[R_MUC], K_EVEN);
    /* central gradients on the interior and the first ghost layer */
    for (int v = 0; v < NREC; v++)
        for (int j = -1; j <= ny; j++)
            for (int i = -1; i <= nx; i++) {
                int c = IX(s, i, j);
                s->gx[v][c] = (s->val[v][IX(s, i + 1, j)] - s->val[v][IX(s, i - 1, j)]) / (2.0 * dx);
                s->gy[v][c] = (s->val[v][IX(s, i, j + 1)] - s->val[v][IX(s, i, j - 1)]) / (2.0 * dx);
            }
}

/* ------------------------------------------------------------ face flux */

/* Literal LBFS flux at the face between cells L and R (padded indices); the unit normal
   n points from L to R along the given axis. F = (He, p, Mx, My, C) normal fluxes. */
static void face_flux(const orc_sim* s, int axis, int cL, int cR, double F[5])
{
    const double dts = s->p.dt_stream, hdx = 0.5 * s->p.dx;
    const double nx_ = axis == 0 ? 1.0 : 0.0, ny_ = axis == 1 ? 1.0 : 0.0;
    double rec[NREC][9];
    /* Eq. 44: reconstruction at x_f - e_a delta_t from the upwind cell */
    for (int a = 0; a < 9; a++) {
        double en = EX[a] * nx_ + EY[a] * ny_;
        double oLx = hdx * nx_ - EX[a] * dts, oLy = hdx * ny_ - EY[a] * dts;
        double oRx = -hdx * nx_ - EX[a] * dts, oRy = -hdx * ny_ - EY[a] * dts;
        for (int v = 0; v < NREC; v++) {
            double vl = s->val[v][cL] + oLx * s->gx[v][cL] + oLy * s->gy[v][cL];
            double vr = s->val[v][cR] + oRx * s->gx[v][cR] + oRy * s->gy[v][cR];
            rec[v][a] = en > 0.0 ? vl : (en < 0.0 ? vr : 0.5 * (vl + vr));
        }
    }
    double rho_f = rec[R_RHO][0], muc_f = rec[R_MUC][0];
    double mu_f = 0.5 * (s->mu[cL] + s->mu[cR]);
    double lam_f = 0.5 * (s->lam[cL] + s->lam[cR]);
    double cp_f = 0.5 * (s->cp[cL] + s->cp[cR]);
    double tau_f = 0.5 + mu_f / (rho_f * CS2 * dts);                 /* Sec. 3.3 */
    double tau_h = 0.5 + lam_f / (rho_f * s->cpref * CS2 * dts);     /* Sec. 3.2 */
    double tau_g = s->p.tau_g;

    /* equilibria at the surrounding points (Eqs. 20, 28, 29 and f^{eq-m}) */
    double fa[9], fm[9], ga[9], ha[9];
    for (int a = 0; a < 9; a++) {
        double u = rec[R_U][a], v = rec[R_V][a];
        fa[a] = f_eq(a, rec[R_P][a], rec[R_RHO][a], u, v);
        fm[a] = f_eq(a, rec[R_P][a], rho_f, u, v);
        ga[a] = g_eq(s, a, rec[R_C][a], rec[R_MUC][a], u, v);
        ha[a] = h_eq(s->cpref, a, rec[R_HE][a], rec[R_T][a], cp_f, u, v);
    }
    /* Eq. 45: macroscopic state at the face */
    double p_f = 0, jx = 0, jy = 0, C_f = 0, He_f = 0;
    for (int a = 0; a < 9; a++) {
        p_f += fa[a]; jx += EX[a] * fa[a]; jy += EY[a] * fa[a];
        C_f += ga[a]; He_f += ha[a];
    }
    double u_f = jx / (rho_f * CS2), v_f = jy / (rho_f * CS2);
    double T_f, Fl_f;
    orc_enthalpy_state(&s->p, He_f, C_f, &T_f, &Fl_f);

    /* face equilibria, non-equilibrium parts and star distributions
       (Eqs. 15-16, 21-22, 30-33 with the viscous sign) */
    double sf[9], sg[9], sh[9], fx0[9];
    for (int a = 0; a < 9; a++) {
        double fe = f_eq(a, p_f, rho_f, u_f, v_f);
        double ge = g_eq(s, a, C_f, muc_f, u_f, v_f);
        double he = h_eq(s->cpref, a, He_f, T_f, cp_f, u_f, v_f);
        double fneq = -tau_f * (fe - fm[a]);
        double gneq = -tau_g * (ge - ga[a]);
        double hneq = -tau_h * (he - ha[a]);
        fx0[a] = fe;
        sf[a] = fe + (1.0 - 1.0 / (2.0 * tau_f)) * fneq;
        sg[a] = ge + (1.0 - 1.0 / (2.0 * tau_g)) * gneq;
        sh[a] = he + (1.0 - 1.0 / (2.0 * tau_h)) * hneq;
    }
    /* Eqs. 40 and 43: normal fluxes */
    double Fp = 0, Fmx = 0, Fmy = 0, Fhe = 0, Fc = 0;
    for (int a = 0; a < 9; a++) {
        double en = EX[a] * nx_ + EY[a] * ny_;
        Fp += en * fx0[a];
        Fmx += en * EX[a] * sf[a];
        Fmy += en * EY[a] * sf[a];
        Fhe += en * sh[a];
        Fc += en * sg[a];
    }
    F[ORC_HE] = Fhe; F[ORC_P] = Fp; F[ORC_MX] = Fmx; F[ORC_MY] = Fmy; F[ORC_C] = Fc;
}

/* Wall faces: no mass and no order-parameter flux; heat conducted through the half
   cell to a fixed-temperature wall, none through an adiabatic one. side = -1 when the
   wall is on the low side of the cell, +1 on the high side. */
static void wall_override(const orc_sim* s, int wall, int c, int side, double F[5])
{
    F[ORC_P] = 0.0;
    F[ORC_C] = 0.0;
    if (s->p.tbc[wall] == 1) {
        double k = s->lam[c] / s->val[R_RHO][c];
        double Tc = s->val[R_T][c], Tw = s->p.tval[wall];
        /* normal flux along +axis: -k dT/dx over the half cell */
        F[ORC_HE] = side < 0 ? -k * (Tc - Tw) / (0.5 * s->p.dx) : -k * (Tw - Tc) / (0.5 * s->p.dx);
    } else {
        F[ORC_HE] = 0.0;
    }
}

static void all_fluxes(orc_sim* s)
{
    int nx = s->nx, ny = s->ny;
    double F[5];
    for (int j = 0; j < ny; j++)
        for (int i = 0; i <= nx; i++) {
            face_flux(s, 0, IX(s, i - 1, j), IX(s, i, j), F);
            if (!s->p.periodic[0] && i == 0) wall_override(s, 0, IX(s, 0, j), -1, F);
            if (!s->p.periodic[0] && i == nx) wall_override(s, 1, IX(s, nx - 1, j), +1, F);
            for (int k = 0; k < 5; k++) s->fx[k][j * (nx + 1) + i] = F[k];
        }
    for (int j = 0; j <= ny; j++)
        for (int i = 0; i < nx; i++) {
            face_flux(s, 1, IX(s, i, j - 1), IX(s, i, j), F);
            if (!s->p.periodic[1] && j == 0) wall_override(s, 2, IX(s, i, 0), -1, F);
            if (!s->p.periodic[1] && j == ny) wall_override(s, 3, IX(s, i, ny - 1), +1, F);
            for (int k = 0; k < 5; k++) s->fy[k][j * nx + i] = F[k];
        }
}

/* R(W) of Eqs. 42 and 46 with the sources of Eq. 41 */
static void rhs(orc_sim* s, double* const Win[5], double* const Rout[5])
{
    int nx = s->nx, ny = s->ny;
    double dx = s->p.dx;
    double vc = 1.0 - s->p.rho[0] / s->p.rho[1];   /* 1 - rho_s / rho_l */
    primitives(s, Win);
    all_fluxes(s);
    double* u = s->val[R_U]; double* v = s->val[R_V];
    double* rho = s->val[R_RHO]; double* muc = s->val[R_MUC];
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            int c = IX(s, i, j);
            int E = IX(s, i + 1, j), Wc = IX(s, i - 1, j), N = IX(s, i, j + 1), Sc = IX(s, i, j - 1);
            double divu = (u[E] - u[Wc]) / (2.0 * dx) + (v[N] - v[Sc]) / (2.0 * dx);
            double drx = (rho[E] - rho[Wc]) / (2.0 * dx), dry = (rho[N] - rho[Sc]) / (2.0 * dx);
            double dmx = (muc[E] - muc[Wc]) / (2.0 * dx), dmy = (muc[N] - muc[Sc]) / (2.0 * dx);
            double Cc = s->val[R_C][c], r = rho[c];
            double src[5];
            src[ORC_HE] = s->cp[c] * s->val[R_T][c] * divu;
            src[ORC_P] = CS2 * (u[c] * drx + v[c] * dry) + r * CS2 * vc * s->S[c];
            src[ORC_MX] = CS2 * (-Cc * dmx + s->fmg[0][c] + r * s->p.grav[0] - r * u[c] * s->fs[c] / s->p.dt);
            src[ORC_MY] = CS2 * (-Cc * dmy + s->fmg[1][c] + r * s->p.grav[1] - r * v[c] * s->fs[c] / s->p.dt);
            src[ORC_C] = Cc * vc * s->S[c];
            for (int k = 0; k < 5; k++) {
                double div = (s->fx[k][j * (nx + 1) + i + 1] - s->fx[k][j * (nx + 1) + i] +
                              s->fy[k][(j + 1) * nx + i] - s->fy[k][j * nx + i]) / dx;
                Rout[k][c] = -div + src[k];
            }
        }
}

/* ------------------------------------------------------------------ API */

int orc_init(orc_sim* s)
{
    const orc_params* p = &s->p;
    double dx = p->dx;
    for (int j = 0; j < s->ny; j++)
        for (int i = 0; i < s->nx; i++) {
            int c = IX(s, i, j);
            double x = (i + 0.5) * dx, y = (j + 0.5) * dx;
            double C;
            if (p->init_kind == 0) {
                double r = sqrt((x - p->drop_cx) * (x - p->drop_cx) + (y - p->drop_cy) * (y - p->drop_cy));
                C = 0.5 * (1.0 + tanh(2.0 * (p->drop_r - r) / p->xi));
            } else {
                C = p->c_init;
            }
            double ct = clamp01(C);
            double cp_sol = ct * p->cp[0] + (1.0 - ct) * p->cp[2];
            double cp_liq = ct * p->cp[1] + (1.0 - ct) * p->cp[2];
            /* inverse of Eq. 8 at T_init */
            double Ts = p->t_melt, Tl = p->t_liquidus, He;
            if (p->t_init >= Tl)
                He = cp_liq * p->t_init + ct * p->latent;
            else if (p->t_init >= Ts)   /* only when Ts < Tl */
                He = cp_sol * Ts + (p->t_init - Ts) / (Tl - Ts) * (cp_liq * Tl + ct * p->latent - cp_sol * Ts);
            else
                He = cp_sol * p->t_init;
            s->W[ORC_HE][c] = He;
            s->W[ORC_P][c] = 0.0;
            s->W[ORC_MX][c] = 0.0;
            s->W[ORC_MY][c] = 0.0;
            s->W[ORC_C][c] = C;
            s->S[c] = 0.0;
            s->phi[c] = phi_applied(s, x, y);
        }
    /* converge the magnetic potential (Table 1, before the main loop) */
    compute_mum(s);
    double r0 = orc_mag_residual(s);
    double om = p->init_omega;
    if (om <= 0.0) {
        int nmax = s->nx > s->ny ? s->nx : s->ny;
        om = 2.0 / (1.0 + sin(M_PI / nmax));
    }
    int used = 0;
    int check = p->init_check > 0 ? p->init_check : 50;
    double r = r0;
    while (r0 > 0.0 && used < p->init_max && r > p->init_tol * r0) {
        int k = check;
        if (used + k > p->init_max) k = p->init_max - used;
        for (int q = 0; q < k; q++) { rb_pass(s, 0, om); rb_pass(s, 1, om); }
        used += k;
        r = orc_mag_residual(s);
    }
    s->res = r;
    s->t = 0.0; s->step = 0.0;
    double vol = 0.0;
    for (int j = 0; j < s->ny; j++)
        for (int i = 0; i < s->nx; i++) vol += clamp01(s->W[ORC_C][IX(s, i, j)]) * dx * dx;
    s->vol0 = vol;
    kelvin(s);
    return used;
}

/* The magnetic update of one time step: `sweeps` iterations of the chosen method, or,
   with mag_max_iters > 0, chunks of `sweeps` iterations until the residual reaches
   mag_tol (checked after every chunk) or mag_max_iters iterations are done. */
static double mag_phase(orc_sim* s)
{
    const orc_params* p = &s->p;
    int used = 0;
    double r;
    for (;;) {
        r = p->mag_method == 1 ? orc_mag_lbfs(s, p->sweeps, p->mag_lbfs_d, p->mag_lbfs_dtau)
                               : orc_mag_sweeps(s, p->sweeps, p->omega);
        used += p->sweeps;
        if (p->mag_max_iters <= 0 || p->sweeps <= 0 || r <= p->mag_tol || used >= p->mag_max_iters) break;
    }
    return r;
}

void orc_step(orc_sim* s, int nsteps)
{
    int nx = s->nx, ny = s->ny;
    double dt = s->p.dt;
    for (int n = 0; n < nsteps; n++) {
        /* magnetic potential: red-black sweeps or LBFS pseudo-time steps, then the Kelvin
           force (frozen over the stages) */
        s->res = mag_phase(s);
        kelvin(s);
        /* SSP-RK3 on (He, p, Mx, My, C) */
        rhs(s, s->W, s->R);
        for (int k = 0; k < 5; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) {
                    int c = IX(s, i, j);
                    s->Wa[k][c] = s->W[k][c] + dt * s->R[k][c];
                }
        rhs(s, s->Wa, s->R);
        for (int k = 0; k < 5; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) {
                    int c = IX(s, i, j);
                    s->Wb[k][c] = 0.75 * s->W[k][c] + 0.25 * (s->Wa[k][c] + dt * s->R[k][c]);
                }
        rhs(s, s->Wb, s->R);
        /* Table 1 (d): Eq. 8 after the step; lagged dFs/dt for the next step */
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                int c = IX(s, i, j);
                double T0, Fl0, T1, Fl1;
                orc_enthalpy_state(&s->p, s->W[ORC_HE][c], s->W[ORC_C][c], &T0, &Fl0);
                for (int k = 0; k < 5; k++)
                    s->W[k][c] = s->W[k][c] / 3.0 + 2.0 / 3.0 * (s->Wb[k][c] + dt * s->R[k][c]);
                orc_enthalpy_state(&s->p, s->W[ORC_HE][c], s->W[ORC_C][c], &T1, &Fl1);
                s->S[c] = -clamp01(s->W[ORC_C][c]) * (Fl1 - Fl0) / dt;
            }
        s->t += dt;
        s->step += 1.0;
    }
}

void orc_rhs(orc_sim* s, double* Rout)
{
    kelvin(s);
    rhs(s, s->W, s->R);
    int nx = s->nx, ny = s->ny;
    for (int k = 0; k < 5; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) Rout[(size_t)k * nx * ny + j * nx + i] = s->R[k][IX(s, i, j)];
}

void orc_face_fluxes(orc_sim* s, double* fx, double* fy)
{
    primitives(s, s->W);
    all_fluxes(s);
    int nx = s->nx, ny = s->ny;
    size_t nfx = (size_t)(nx + 1) * ny, nfy = (size_t)nx * (ny + 1);
    for (int k = 0; k < 5; k++) {
        memcpy(fx + k * nfx, s->fx[k], nfx * sizeof(double));
        memcpy(fy + k * nfy, s->fy[k], nfy * sizeof(double));
    }
}

void orc_face_inputs(orc_sim* s, double* out)
{
    primitives(s, s->W);
    int nx = s->nx, ny = s->ny;
    size_t n = (size_t)nx * ny;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            int c = IX(s, i, j);
            size_t o = (size_t)j * nx + i;
            for (int v = 0; v < NREC; v++) {
                out[(size_t)v * n + o] = s->val[v][c];
                out[(size_t)(NREC + v) * n + o] = s->gx[v][c];
                out[(size_t)(2 * NREC + v) * n + o] = s->gy[v][c];
            }
            out[(size_t)(3 * NREC) * n + o] = s->mu[c];
            out[(size_t)(3 * NREC + 1) * n + o] = s->lam[c];
            out[(size_t)(3 * NREC + 2) * n + o] = s->cp[c];
        }
}

void orc_get(orc_sim* s, int field, double* out)
{
    int nx = s->nx, ny = s->ny;
    if (field == ORC_MUC) primitives(s, s->W);
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            int c = IX(s, i, j);
            double v = 0.0, T, Fl;
            switch (field) {
            case ORC_HE: case ORC_P: case ORC_MX: case ORC_MY: case ORC_C: v = s->W[field][c]; break;
            case ORC_PHI: v = s->phi[c]; break;
            case ORC_S: v = s->S[c]; break;
            case ORC_T: orc_enthalpy_state(&s->p, s->W[ORC_HE][c], s->W[ORC_C][c], &T, &Fl); v = T; break;
            case ORC_FL: orc_enthalpy_state(&s->p, s->W[ORC_HE][c], s->W[ORC_C][c], &T, &Fl); v = Fl; break;
            case ORC_FMGX: v = s->fmg[0][c]; break;
            case ORC_FMGY: v = s->fmg[1][c]; break;
            case ORC_MUC: v = s->val[R_MUC][c]; break;
            default: break;
            }
            out[j * nx + i] = v;
        }
}

void orc_set(orc_sim* s, int field, const double* in)
{
    int nx = s->nx, ny = s->ny;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            int c = IX(s, i, j);
            double v = in[j * nx + i];
            if (field >= ORC_HE && field <= ORC_C) s->W[field][c] = v;
            else if (field == ORC_PHI) s->phi[c] = v;
            else if (field == ORC_S) s->S[c] = v;
        }
}

void orc_set_time(orc_sim* s, double t, double step) { s->t = t; s->step = step; }

void orc_wall_heat_profile(orc_sim* s, double* q)
{
    int nx = s->nx;
    double dx = s->p.dx, tw = s->p.tval[2];
    int on = !s->p.periodic[1] && s->p.tbc[2] == 1;
    for (int i = 0; i < nx; i++) {
        q[i] = 0.0;
        if (!on) continue;
        int c0 = IX(s, i, 0), c1 = IX(s, i, 1);
        double T0, T1, Fl0, Fl1;
        orc_enthalpy_state(&s->p, s->W[ORC_HE][c0], s->W[ORC_C][c0], &T0, &Fl0);
        orc_enthalpy_state(&s->p, s->W[ORC_HE][c1], s->W[ORC_C][c1], &T1, &Fl1);
        double ct = clamp01(s->W[ORC_C][c0]);
        double lam = mix3(s->p.lam, ct * (1.0 - Fl0), ct);
        /* T(y) through (0, Tw), (dx/2, T0), (3dx/2, T1): T'(0) = (9 T0 - T1 - 8 Tw) / (3 dx) */
        q[i] = -lam * (9.0 * T0 - T1 - 8.0 * tw) / (3.0 * dx);
    }
}

void orc_observe(orc_sim* s, orc_obs* o)
{
    int nx = s->nx, ny = s->ny;
    double dx = s->p.dx;
    double sc = 0, scfl = 0, sfs = 0, umax = 0, udrop = 0, nonfinite = 0, heat = 0;
    int ic = (int)floor(s->p.drop_cx / dx);
    if (ic < 0) ic = 0;
    if (ic > nx - 1) ic = nx - 1;
    double height = 0.0, solid_height = 0.0;
    double mx = 0, my = 0, mxx = 0, myy = 0, mxy = 0;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            int c = IX(s, i, j);
            for (int k = 0; k < 5; k++)
                if (!isfinite(s->W[k][c])) nonfinite = 1;
            double C = s->W[ORC_C][c], ct = clamp01(C), T, Fl;
            double x = (i + 0.5) * dx, y = (j + 0.5) * dx;
            mx += ct * x; my += ct * y; mxx += ct * x * x; myy += ct * y * y; mxy += ct * x * y;
            orc_enthalpy_state(&s->p, s->W[ORC_HE][c], C, &T, &Fl);
            double fs = ct * (1.0 - Fl);
            double rho = mix3(s->p.rho, fs, ct);
            double u = s->W[ORC_MX][c] / (rho * CS2), v = s->W[ORC_MY][c] / (rho * CS2);
            double um = sqrt(u * u + v * v);
            sc += ct; scfl += ct * Fl; sfs += fs;
            if (um > umax) umax = um;
            if (ct >= 0.5 && um > udrop) udrop = um;
            if (i == ic) {
                height += ct * dx;
                solid_height += fs * dx;
            }
            if (j == 0 && !s->p.periodic[1] && s->p.tbc[2] == 1) {
                double lam = mix3(s->p.lam, fs, ct);
                heat += -lam * (T - s->p.tval[2]) / (0.5 * dx) * dx;
            }
        }
    o->t = s->t; o->step = s->step;
    o->volume = sc * dx * dx;
    o->volume0 = s->vol0;
    o->liquid_fraction = sc > 0 ? scfl / sc : 0.0;
    o->solid_ratio = s->vol0 > 0 ? sfs * dx * dx / s->vol0 : 0.0;
    o->mag_residual = s->res;
    o->umax = umax;
    o->nonfinite = nonfinite;
    o->height = height;
    o->solid_height = solid_height;
    o->umax_drop = udrop;
    o->wall_heat = heat;
    /* Eq. 50 with the liquid properties and the initial radius R0 */
    double alpha_l = s->p.lam[1] / (s->p.rho[1] * s->p.cp[1]);
    o->fourier = alpha_l * s->t / (s->p.drop_r * s->p.drop_r);
    o->peclet = udrop * 2.0 * s->p.drop_r / alpha_l;
    /* shape: covariance of the Ct distribution; an ellipse of semi-axes a, b has the
       variance a^2/4 along its axis a */
    o->centroid_x = o->centroid_y = o->semi_axis_x = o->semi_axis_y = 0.0;
    o->semi_axis_major = o->semi_axis_minor = o->major_axis_deg = 0.0;
    if (sc > 0.0) {
        double cx = mx / sc, cy = my / sc;
        double vxx = mxx / sc - cx * cx, vyy = myy / sc - cy * cy, vxy = mxy / sc - cx * cy;
        if (vxx < 0.0) vxx = 0.0;
        if (vyy < 0.0) vyy = 0.0;
        double mean = 0.5 * (vxx + vyy), dev = sqrt(0.25 * (vxx - vyy) * (vxx - vyy) + vxy * vxy);
        double lmin = mean - dev > 0.0 ? mean - dev : 0.0;
        o->centroid_x = cx; o->centroid_y = cy;
        o->semi_axis_x = 2.0 * sqrt(vxx); o->semi_axis_y = 2.0 * sqrt(vyy);
        o->semi_axis_major = 2.0 * sqrt(mean + dev); o->semi_axis_minor = 2.0 * sqrt(lmin);
        double ang = 0.5 * atan2(2.0 * vxy, vxx - vyy) * 180.0 / M_PI;
        if (ang <= -90.0) ang += 180.0;
        o->major_axis_deg = ang;
    }
}

/*
 * lbfs_oracle.h -- plain FP64 CPU oracle of the enthalpy-based lattice Boltzmann
 * flux solver (LBFS) for a freezing ferrofluid droplet in a uniform magnetic field
 * (Zhou, Yang, Wang, Wu, Niu, arXiv 2511.10257).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load this library. It shares no code, header, table or helper
 * with the HIP product library; the two are independent implementations of the
 * same readings of the paper.
 *
 * Units: lattice units with c = 1, cs^2 = 1/3; dx is a parameter (cell size).
 * Grid: nx * ny square cells, cell (i,j) centred at ((i+1/2)dx, (j+1/2)dx).
 * Walls are numbered 0 = west (x=0), 1 = east (x=nx*dx), 2 = south (y=0),
 * 3 = north (y=ny*dx).
 */
#ifndef LBFS_ORACLE_H
#define LBFS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* conserved fields, Eq. 39 without the magnetic potential (which is relaxed, not
   time-integrated): total enthalpy, pressure, rho*cs^2*u, rho*cs^2*v, order parameter */
enum { ORC_HE = 0, ORC_P = 1, ORC_MX = 2, ORC_MY = 3, ORC_C = 4,
       ORC_PHI = 5,   /* magnetic scalar potential phi_m (Eq. 3)                     */
       ORC_S = 6,     /* lagged dFs/dt used by the volume-change sources (Eqs. 9-10)  */
       ORC_T = 7,     /* temperature, Eq. 8 (read only)                               */
       ORC_FL = 8,    /* liquid fraction, Eq. 8 (read only)                           */
       ORC_FMGX = 9, ORC_FMGY = 10, /* Kelvin force of the last step, Eq. 6 (read only) */
       ORC_MUC = 11,  /* chemical potential (read only, from the current C)           */
       ORC_NFIELDS = 12 };

typedef struct orc_params {
    int nx, ny;
    double dx;            /* cell size                                     */
    double dt;            /* Runge-Kutta time step                         */
    double dt_stream;     /* streaming step delta_t of the local LBE       */
    double rho[3], mu[3], cp[3], lam[3], chi[3];  /* [solid, liquid, gas]  */
    double latent;        /* latent heat L                                 */
    double t_melt;        /* Ts = Tl = Tm                                  */
    double t_init;        /* initial temperature                           */
    double mu0, h0, angle_deg;   /* vacuum permeability, applied field, direction */
    double grav[2];
    double sigma, xi;     /* interfacial tension, interface thickness      */
    double mobility;      /* M_c                                           */
    double tau_g;         /* relaxation parameter of the phase field       */
    double drop_cx, drop_cy, drop_r;
    int init_kind;        /* 0: droplet (tanh profile), 1: uniform C = c_init */
    double c_init;
    int periodic[2];      /* x, y                                          */
    int tbc[4];           /* thermal wall: 0 adiabatic, 1 fixed temperature */
    double tval[4];
    int mbc[4];           /* magnetic wall: 0 insulating, 1 fixed potential of the applied field */
    int sweeps;           /* red-black sweeps per time step                */
    double omega;         /* relaxation factor of the per-step sweeps      */
    double init_omega;    /* SOR factor of the initial solve (<=0: automatic) */
    double init_tol;      /* relative residual target of the initial solve */
    int init_max;         /* sweep cap of the initial solve                */
    int init_check;       /* sweeps between residual checks                */
    int mag_method;       /* per-step magnetic update: 0 red-black sweeps of the compact
                             system, 1 LBFS pseudo-time solve of Eq. 17 (Sec. 3.1), both
                             `sweeps` iterations per time step                          */
    double mag_lbfs_d;    /* free parameter D of tau_m (Sec. 3.1), > 0                   */
    double mag_lbfs_dtau; /* pseudo-time step (<= 0: dx^2 / (4 D mu_max))                */
    int mag_max_iters;    /* > 0: repeat chunks of `sweeps` iterations until ||r||_2 <=
                             mag_tol, at most this many iterations per step; 0: exactly
                             `sweeps` iterations per step                               */
    double mag_tol;       /* absolute target of ||r||_2 for mag_max_iters > 0            */
    double contact_angle[4]; /* wetting walls: contact angle through the liquid (degrees,
                                0 < theta < 180; 90 is the mirror condition)             */
    double t_liquidus;    /* Tl >= t_melt (the solidus Ts) of Eq. 8                      */
} orc_params;

typedef struct orc_obs {
    double t, step;
    double liquid_fraction;  /* sum(Ct*Fl)/sum(Ct)                         */
    double solid_ratio;      /* Q_L of Eq. 51: sum(Fs dA)/A0               */
    double volume, volume0;  /* sum(Ct dA) now and at initialisation       */
    double mag_residual;     /* ||r||_2 of the magnetic system after the sweeps */
    double umax;             /* max |u| over all cells                     */
    double nonfinite;        /* 1 if any conserved value is not finite     */
    double height;           /* sum(Ct dx) along the column through drop_cx */
    double umax_drop;        /* max |u| over cells with Ct >= 1/2          */
    double wall_heat;        /* integrated heat flux into the south wall   */
    double fourier;          /* Fo of Eq. 50: lambda_l t / (rho_l Cp_l R0^2) */
    double peclet;           /* Pe of Eq. 50, read as umax_drop D / alpha_l,
                                D = 2 R0, alpha_l = lambda_l / (rho_l Cp_l) */
    double centroid_x, centroid_y;        /* Ct-weighted centroid                   */
    double semi_axis_x, semi_axis_y;      /* 2 sqrt(Ct-weighted variance) along x, y */
    double semi_axis_major, semi_axis_minor, major_axis_deg;  /* principal axes   */
    double solid_height;     /* sum(Fs dx) along the column through drop_cx: the frozen
                                part of the droplet's height there (Fig. 17 reading) */
} orc_obs;

typedef struct orc_sim orc_sim;

/* Eq. 50 conversions: L = Cp_l (Tm - Tw) / Ste and H0 = sqrt(Bo_m sigma / (mu0 D)),
   with D the droplet diameter. */
void orc_params_from_dimless(orc_params* p, double ste, double t_wall, double bo_m);

orc_sim* orc_new(const orc_params* p);      /* NULL on invalid parameters */
void orc_free(orc_sim* s);
int orc_init(orc_sim* s);                    /* initial fields + converged magnetic solve; returns sweeps used */
void orc_step(orc_sim* s, int nsteps);
void orc_rhs(orc_sim* s, double* R);         /* R(W) of Eq. 46 for the current state; R is 5*nx*ny, field-major */
void orc_face_fluxes(orc_sim* s, double* fx, double* fy); /* fx: 5*(nx+1)*ny, fy: 5*nx*(ny+1) */
/* The inputs of the face fluxes for the current state, per cell (nx*ny each, row-major):
   the eight reconstructed variables p, u, v, rho, C, mu_c, T, He, their central x and y
   gradients (8 + 8 blocks), then mu, lambda and Cp of Eq. 11; 27*nx*ny values. */
void orc_face_inputs(orc_sim* s, double* out);
void orc_get(orc_sim* s, int field, double* out);          /* nx*ny, row-major (j*nx+i) */
void orc_set(orc_sim* s, int field, const double* in);
void orc_set_time(orc_sim* s, double t, double step);
void orc_observe(orc_sim* s, orc_obs* o);
double orc_mag_sweeps(orc_sim* s, int nsweeps, double omega);  /* returns ||r||_2 after */
double orc_mag_residual(orc_sim* s);
/* LBFS pseudo-time solve of the magnetic potential (Eqs. 12-18): permeability from
   the current state, then nsteps SSP-RK3 steps of size dtau (<= 0: automatic) of
   Eq. 17 with the face fluxes built from m* (Eq. 16); returns ||r||_2 after. */
double orc_mag_lbfs(orc_sim* s, int nsteps, double D, double dtau);
/* Normal face fluxes sum_a e_a.n m*_a of the current potential (Eq. 18): fx is
   (nx+1)*ny (x-faces, row-major j*(nx+1)+i, face i between cells i-1 and i), fy is
   nx*(ny+1); the permeability is taken from the current state. */
void orc_mag_lbfs_fluxes(orc_sim* s, double D, double* fx, double* fy);
/* the automatic pseudo-time step of orc_mag_lbfs */
double orc_mag_lbfs_dtau(const orc_params* p, double D);

/* Local heat flux Q = -lambda dT/dy on the south wall (Sec. 5.2, Fig. 15), one value
   per column: the second-order one-sided difference through the wall temperature and
   the first two cell centres, lambda of the wall cell (Eq. 11). Zero when the south
   wall is not a fixed-temperature wall. q holds nx values. */
void orc_wall_heat_profile(orc_sim* s, double* q);

/* pointwise pieces, exposed for the moment and branch pins */
void orc_lattice(double* ex, double* ey, double* w);
void orc_enthalpy_state(const orc_params* p, double He, double C, double* T, double* Fl);
void orc_equilibria(const orc_params* p, double pr, double rho, double u, double v,
                    double C, double muc, double He, double T, double cp,
                    double* feq, double* geq, double* heq);

#ifdef __cplusplus
}
#endif
#endif

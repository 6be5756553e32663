// lbfs_face.hpp -- the LBFS flux through one face, and the Eq. 8 enthalpy map it uses.
//
// Written for the device (the stage kernels include it) and for the host in FP64, where
// a CPU test runs it on the face inputs of the oracle and compares the fluxes with the
// oracle's literal nine-point procedure. The FP32 reciprocals use the hardware
// instruction and exist on the device only.
#pragma once

#include "lbfs_internal.hpp"

namespace lbfs {

#define LBFS_HD __host__ __device__ __forceinline__

template <typename T>
LBFS_HD T clamp01(T c) { return c < T(0) ? T(0) : (c > T(1) ? T(1) : c); }

// 1 / x for x bounded away from 0 and infinity (densities): the hardware reciprocal
// (1 ulp) in FP32, a correctly rounded division in FP64
__device__ __forceinline__ float rcp_bounded(float x) { return __builtin_amdgcn_rcpf(x); }
LBFS_HD double rcp_bounded(double x) { return 1.0 / x; }

// num / den of the Eq. 8 branch. The denominators are heat capacities (>= the gas one)
// or, on the mushy branch, Ct L, which is tiny in a trace of liquid; there the quotient
// is a liquid fraction in [0, 1], clamped by the caller. FP32: the hardware reciprocal
// of the denominator raised to the smallest normal float (1 ulp), FP64: a correctly
// rounded division.
__device__ __forceinline__ float branch_quotient(float num, float den)
{
    return num * __builtin_amdgcn_rcpf(fmaxf(den, 1.17549435e-38f));
}
LBFS_HD double branch_quotient(double num, double den) { return num / den; }

// Eq. 8 with solidus Ts and liquidus Tl, local latent heat Ct L and branch heat
// capacities of the solid-gas and liquid-gas mixtures
template <typename T>
LBFS_HD void enthalpy_state(const Coef<T>& K, T He, T C, T& Tt, T& Fl)
{
    const T ct = clamp01(C);
    const T cps = ct * K.cp[0] + (T(1) - ct) * K.cp[2];
    const T cpl = ct * K.cp[1] + (T(1) - ct) * K.cp[2];
    const T ts = K.tm, tl = K.tl;
    const T Hes = cps * ts;
    const T Hel = cpl * tl + ct * K.latent;
    // branch of Eq. 8, then the one quotient that branch needs
    const bool liq = He > Hel;
    const bool mushy = !liq && He >= Hes && Hel > Hes;
    const T num = liq ? He - Hel : (mushy ? He - Hes : He);
    const T den = liq ? cpl : (mushy ? Hel - Hes : cps);
    const T q = branch_quotient(num, den);
    Fl = liq ? T(1) : (mushy ? clamp01(q) : T(0));
    Tt = liq ? tl + q : (mushy ? ts + Fl * (tl - ts) : q);
}

// Inputs of one side of a face, in the face frame (n = normal from L to R,
// t = tangential): values and (d/dn, d/dt) of p, u_n, u_t, rho, C, mu_c, T, He.
enum { V_P = 0, V_UN, V_UT, V_RHO, V_C, V_MUC, V_T, V_HE, NV };

template <typename T>
struct Side {
    T v[NV], gn[NV], gt[NV];
    T mu, lam, cp;
};

// LBFS fluxes through one face with delta_t = dx/2 (h = dx/2). The nine points
// x_f - e_a delta_t of Eq. 44 are the two cell centres (a with e_n = +-1, e_t = 0),
// points on the cell axes half a cell off the face line (diagonals) and points on
// the face line (e_n = 0, averaged over both sides). The flux is evaluated as
// moments: with Gamma_a = e.u + 1.5 (e.u)^2 - 0.5 u^2,
//   f_eq,a = w (p + rho Gamma), f_eqm,a = w (p + rho_f Gamma)   (Eq. 28, f^{eq-m})
//   g_eq,a = w 3 (Q mu_c + C e.u)  (a > 0)                      (Eq. 29)
//   h_eq,a = w (Cp_ref T + 3 Cp_f T Gamma) (+ He - Cp_ref T at a = 0)   (Eq. 20)
// Eq. 45 gives the face state; the star distributions (Eqs. 16, 22, 32, 33 with the
// viscous sign) give F = (3/2 - tau) M_eq(face) + (tau - 1/2) M(surrounding), where
// M_eq(face) are the closed-form moments of the face equilibria (D2Q9 identities).
// The terms linear in p, mu_c and T are summed over the nine points in closed form
// (the points are linear reconstructions, so their weighted sums are combinations of
// the two sides' values and gradients); the terms in Gamma and C e.u are summed point
// by point: those of each side's own three points (its cell centre and two diagonals)
// from that side's values alone (side_part), then those of the face line.
// Output: F[0] He, F[1] p, F[2] normal momentum, F[3] tangential momentum, F[4] C.
// What one side of a face contributes, computed from that side alone: its axis point
// (the cell centre, e = (sgn, 0)) and its two diagonal points (v -+ h dv/dt, e =
// (sgn, +-1)), summed with their weights, and the values the rest of the face needs.
// sgn = +1 for L (e_n = +1 points), -1 for R.
template <typename T>
struct SidePart {
    T A, At, G2, Gnt, B, E;   // this side's share of the sums named in face_flux
    T hv[NV];                 // v + sgn h dv/dn (half of the face-centre reconstruction)
    T gt[NV];                 // dv/dt
    T vp, vt, vmu, gnt, gnmu; // p, T, mu_c and the normal gradients of T and mu_c
    T mu, lam, cp;
};

template <typename T, int SGN>
LBFS_HD void side_part(const Coef<T>& K, const Side<T>& S, SidePart<T>& o)
{
#pragma clang fp reassociate(on)
    const T h = T(0.5) * K.dx;
    const T sg = T(SGN);
    const T w1 = T(1.0 / 9.0), w2 = T(1.0 / 36.0);
    const T un = S.v[V_UN], ut = S.v[V_UT];
    // axis point: Gamma = sgn u_n + u_n^2 - u_t^2 / 2
    const T G = un * un + sg * un - T(0.5) * (ut * ut);
    // diagonals P (e_t = +1, at v - h dv/dt) and M (e_t = -1, at v + h dv/dt); with
    // |u|^2 = (e.u)^2 - 2 e_n e_t u_n u_t, Gamma = e.u + (e.u)^2 + e_n e_t u_n u_t
    const T unP = un - h * S.gt[V_UN], utP = ut - h * S.gt[V_UT];
    const T unM = un + h * S.gt[V_UN], utM = ut + h * S.gt[V_UT];
    const T euP = sg * unP + utP, euM = sg * unM - utM;
    const T gP = euP * euP + euP + sg * (unP * utP);
    const T gM = euM * euM + euM - sg * (unM * utM);
    const T rP = S.v[V_RHO] - h * S.gt[V_RHO], rM = S.v[V_RHO] + h * S.gt[V_RHO];
    const T tP = S.v[V_T] - h * S.gt[V_T], tM = S.v[V_T] + h * S.gt[V_T];
    const T cP = S.v[V_C] - h * S.gt[V_C], cM = S.v[V_C] + h * S.gt[V_C];
    const T XP = rP * gP, XM = rM * gM;
    o.A = w1 * (S.v[V_RHO] * G) + w2 * (XP + XM);
    o.At = w2 * (XP - XM);
    o.G2 = w1 * G + w2 * (gP + gM);
    o.Gnt = w2 * (gP - gM);
    o.B = w1 * (S.v[V_T] * G) + w2 * (tP * gP + tM * gM);
    o.E = w1 * (S.v[V_C] * (sg * un)) + w2 * (cP * euP + cM * euM);
#pragma unroll
    for (int k = 0; k < NV; k++) {
        o.hv[k] = S.v[k] + sg * h * S.gn[k];
        o.gt[k] = S.gt[k];
    }
    o.vp = S.v[V_P];
    o.vt = S.v[V_T];
    o.vmu = S.v[V_MUC];
    o.gnt = S.gn[V_T];
    o.gnmu = S.gn[V_MUC];
    o.mu = S.mu;
    o.lam = S.lam;
    o.cp = S.cp;
}

template <typename T>
LBFS_HD void face_flux(const Coef<T>& K, const SidePart<T>& L, const SidePart<T>& R, T F[5])
{
#pragma clang fp reassociate(on)
    const T h = T(0.5) * K.dx;
    const T hh = T(0.5) * h;
    const T w0 = T(4.0 / 9.0), w1 = T(1.0 / 9.0);
    // the face centre (point 0) and the face-line points 2 (e = (0, +1), at m - h gt)
    // and 4 (e = (0, -1), at m + h gt), gt the mean tangential gradient
    auto mid = [&](int k) { return T(0.5) * (L.hv[k] + R.hv[k]); };
    auto dt = [&](int k) { return hh * (L.gt[k] + R.gt[k]); };
    const T un0 = mid(V_UN), ut0 = mid(V_UT), r0 = mid(V_RHO), t0 = mid(V_T), c0 = mid(V_C);
    const T dun = dt(V_UN), dut = dt(V_UT), dr = dt(V_RHO), dtt = dt(V_T), dc = dt(V_C);
    const T un2 = un0 - dun, ut2 = ut0 - dut, un4 = un0 + dun, ut4 = ut0 + dut;
    const T g0 = T(-0.5) * (un0 * un0 + ut0 * ut0);
    const T g2 = ut2 * ut2 + ut2 - T(0.5) * (un2 * un2);
    const T g4 = ut4 * ut4 - ut4 - T(0.5) * (un4 * un4);
    const T X2 = (r0 - dr) * g2, X4 = (r0 + dr) * g4;
    // Sums over the nine points of rho Gamma (A, and times e_n, e_t: An, At), of Gamma
    // times e_n^2 and e_n e_t (G2, Gnt), of T Gamma (B, Bn) and of C e.u (E, En)
    const T A = w0 * (r0 * g0) + w1 * (X2 + X4) + (L.A + R.A);
    const T An = L.A - R.A;
    const T At = w1 * (X2 - X4) + (L.At + R.At);
    const T G2 = L.G2 + R.G2;
    const T Gnt = L.Gnt - R.Gnt;
    const T B = w0 * (t0 * g0) + w1 * ((t0 - dtt) * g2 + (t0 + dtt) * g4) + (L.B + R.B);
    const T Bn = L.B - R.B;
    const T E = w1 * ((c0 - dc) * ut2 - (c0 + dc) * ut4) + (L.E + R.E);
    const T En = L.E - R.E;

    const T rho_f = r0;
    const T irho_f = rcp_bounded(rho_f);
    const T mu_f = T(0.5) * (L.mu + R.mu);
    const T lam_f = T(0.5) * (L.lam + R.lam);
    const T cp_f = T(0.5) * (L.cp + R.cp);
    const T cpref = K.cpref;
    const T Q = K.qg;
    const T tau_f = T(0.5) + mu_f * irho_f * K.tauf_k;
    const T tau_h = T(0.5) + lam_f * irho_f * K.tauh_k;
    const T tau_g = K.tau_g;
    const T c3 = T(3) * cp_f;
    // the parts linear in p, mu_c and T summed in closed form over the nine points
    const T pS = L.vp + R.vp;
    const T S0 = T(2.0 / 3.0) * mid(V_P) + T(1.0 / 6.0) * pS + A;
    const T Sn = T(1.0 / 6.0) * (L.vp - R.vp) + An;
    const T St = -(h * T(1.0 / 6.0)) * (L.gt[V_P] + R.gt[V_P]) + At;
    const T Mnn = T(1.0 / 6.0) * pS + rho_f * G2;
    const T Mnt = (h * T(1.0 / 18.0)) * (R.gt[V_P] - L.gt[V_P]) + rho_f * Gnt;
    const T Hn = (cpref * T(1.0 / 6.0)) * (L.vt - R.vt) + c3 * Bn;
    const T Gn = (T(0.5) * Q) * (L.vmu - R.vmu) + T(3) * En;
    // Eq. 45: face state
    const T p_f = S0;
    const T un_f = T(3) * Sn * irho_f;
    const T ut_f = T(3) * St * irho_f;
    const T C_f = c0 - (Q * hh) * (L.gnmu - R.gnmu) + T(3) * E;
    const T He_f = mid(V_HE) - (cpref * h * T(1.0 / 6.0)) * (L.gnt - R.gnt) + c3 * B;
    T T_f, Fl_f;
    enthalpy_state<T>(K, He_f, C_f, T_f, Fl_f);
    F[1] = Sn;
    F[2] = (T(1.5) - tau_f) * (p_f + rho_f * un_f * un_f) * T(1.0 / 3.0) + (tau_f - T(0.5)) * Mnn;
    F[3] = (T(1.5) - tau_f) * (rho_f * un_f * ut_f) * T(1.0 / 3.0) + (tau_f - T(0.5)) * Mnt;
    F[4] = (T(1.5) - tau_g) * C_f * un_f + (tau_g - T(0.5)) * Gn;
    F[0] = (T(1.5) - tau_h) * cp_f * T_f * un_f + (tau_h - T(0.5)) * Hn;
}

}  // namespace lbfs

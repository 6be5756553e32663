// face_flux_host.cpp -- runs the library's face flux (lbfs_face.hpp) on the host in FP64.
//
// Test infrastructure for tests/test_face_closed_form.py. Reads from stdin: int32 nfaces,
// then 12 doubles of parameters (dx, cpref, qg, tauf_k, tauh_k, tau_g, cp[3], tm, tl,
// latent), then per face two sides of 27 doubles each (values, normal gradients and
// tangential gradients of p, u_n, u_t, rho, C, mu_c, T, He; then mu, lambda, Cp).
// Writes per face the five fluxes (He, p, normal momentum, tangential momentum, C).
#include <cstdint>
#include <cstdio>
#include <vector>

#include "lbfs_face.hpp"

using namespace lbfs;

static bool read_all(void* dst, size_t n) { return fread(dst, 1, n, stdin) == n; }

int main()
{
    int32_t nf = 0;
    double prm[12];
    if (!read_all(&nf, sizeof nf) || nf < 0 || !read_all(prm, sizeof prm)) return 2;
    Coef<double> K{};
    K.dx = prm[0];
    K.cpref = prm[1];
    K.qg = prm[2];
    K.tauf_k = prm[3];
    K.tauh_k = prm[4];
    K.tau_g = prm[5];
    K.cp[0] = prm[6];
    K.cp[1] = prm[7];
    K.cp[2] = prm[8];
    K.tm = prm[9];
    K.tl = prm[10];
    K.latent = prm[11];
    std::vector<double> in(54), out(5);
    for (int f = 0; f < nf; f++) {
        if (!read_all(in.data(), 54 * sizeof(double))) return 3;
        Side<double> S[2];
        for (int k = 0; k < 2; k++) {
            const double* a = in.data() + 27 * k;
            for (int v = 0; v < NV; v++) {
                S[k].v[v] = a[v];
                S[k].gn[v] = a[NV + v];
                S[k].gt[v] = a[2 * NV + v];
            }
            S[k].mu = a[24];
            S[k].lam = a[25];
            S[k].cp = a[26];
        }
        SidePart<double> PL, PR;
        side_part<double, 1>(K, S[0], PL);
        side_part<double, -1>(K, S[1], PR);
        face_flux<double>(K, PL, PR, out.data());
        if (fwrite(out.data(), sizeof(double), 5, stdout) != 5) return 4;
    }
    return 0;
}

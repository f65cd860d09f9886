/*
 * spectra_oracle.c -- TEST INFRASTRUCTURE: plain FP64 CPU reference of the
 * smooth Cooper-Frye spectra (CLVisc, arXiv:1802.04449, Sec. IV, eq.
 * cooper_frye with f_eq and delta f of eqn. feq; App. A.2 parallelises the sum
 * over surface elements on the GPU).
 *
 * Only the test suite may load this code; the HIP library shares none of it.
 *
 * For species s (mass m, degeneracy g, statistics sigma = +1 Fermi-Dirac,
 * -1 Bose-Einstein, 0 Boltzmann, chemical potential mu) and bin (Y, pT, phi):
 *
 *   dN/(dY pT dpT dphi) = g / (2 pi hbarc)^3  sum_elements  p^mu dSigma_mu f (1 + df)
 *
 * with m_T = sqrt(m^2 + pT^2) and, at an element of centre (tau, eta_s):
 *   p~ = (m_T cosh(Y - eta_s), pT cos phi, pT sin phi, m_T sinh(Y - eta_s))
 *   (tilde components: p~^eta = tau p^eta), so that
 *   p^mu dSigma_mu = p~^tau dSigma_tau + p~^x dSigma_x + p~^y dSigma_y + (p~^eta / tau) dSigma_eta
 *   (dSigma_mu in the coordinates (tau, x, y, eta_s), units fm^3),
 *   p.u = p~^tau u~^tau - p~^x u~^x - p~^y u~^y - p~^eta u~^eta,
 *   f = 1 / (exp((p.u - mu)/T) + sigma),
 *   df = (1 - sigma f) p~_mu p~_nu pi~^{mu nu} / (2 T^2 (e + P)), p~_mu = g~_mu mu p~^mu
 *   (df = 0 when e + P is given as 0).
 * Units: masses, momenta, T and mu in GeV, dSigma in fm^3, e + P in GeV/fm^3,
 * pi~ in GeV/fm^3; the result in GeV^-2.
 *
 * Surface element records are those of the finder (24 doubles): [1] tau,
 * [4] eta_s, [5..8] dSigma_mu, [9..11] u~ (x, y, eta), [12..21] pi~.
 * out[((s * nY + iy) * npt + ip) * nphi + iphi].
 */
#include <math.h>

#define HBARC_S 0.1973269804

#include "oracle_mut.h" /* planted-mistake switches (mutant build only) */

int orc_spectra(const double *el, long n, double T, double eps_plus_P, int ns, const double *mass,
                const double *dof, const int *stat, const double *mu, int nY, const double *Y,
                int npt, const double *pt, int nphi, const double *phi, double *out) {
    if (n < 0 || ns < 1 || nY < 1 || npt < 1 || nphi < 1 || !(T > 0)) return -1;
    const double pref = 1.0 / pow(2.0 * M_PI * HBARC_S, 3);
    const double gt[4] = {1.0, -1.0, -1.0, -1.0};
    static const int sym[4][4] = {{0, 1, 2, 3}, {1, 4, 5, 6}, {2, 5, 7, 8}, {3, 6, 8, 9}};
    for (int s = 0; s < ns; ++s)
        for (int iy = 0; iy < nY; ++iy)
            for (int ip = 0; ip < npt; ++ip)
                for (int iq = 0; iq < nphi; ++iq) {
                    const double mT = sqrt(mass[s] * mass[s] + pt[ip] * pt[ip]);
                    double sum = 0.0;
                    for (long e = 0; e < n; ++e) {
                        const double *r = el + e * 24;
                        const double tau = r[1], eta = r[4];
                        const double ux = r[9], uy = r[10], ue = r[11];
                        const double ut = sqrt(1.0 + ux * ux + uy * uy + ue * ue);
                        const double p[4] = {mT * cosh(Y[iy] - eta), pt[ip] * cos(phi[iq]),
                                             pt[ip] * sin(phi[iq]), mT * sinh(Y[iy] - eta)};
                        const double pdS = p[0] * r[5] + p[1] * r[6] + p[2] * r[7] +
                                           (MUT(26) ? p[3] : p[3] / tau) * r[8];
                        const double pu = p[0] * ut - (MUT(27) ? -p[1] : p[1]) * ux - p[2] * uy -
                                          p[3] * ue;
                        const double f = 1.0 / (exp((pu - mu[s]) / T) + (double)stat[s]);
                        double df = 0.0;
                        if (eps_plus_P > 0.0) {
                            double ppi = 0.0;
                            for (int a = 0; a < 4; ++a)
                                for (int b = 0; b < 4; ++b)
                                    ppi += gt[a] * p[a] * gt[b] * p[b] * r[12 + sym[a][b]];
                            df = (MUT(25) ? 1.0 + (double)stat[s] * f : 1.0 - (double)stat[s] * f) *
                                 ppi / (2.0 * T * T * eps_plus_P);
                        }
                        sum += pdS * f * (1.0 + df);
                    }
                    out[((long)(s * nY + iy) * npt + ip) * nphi + iq] = dof[s] * pref * sum;
                }
    return 0;
}

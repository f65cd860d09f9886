/*
 * surface_oracle.c -- TEST INFRASTRUCTURE: plain FP64 CPU reference of the
 * freeze-out hypersurface finder (CLVisc, arXiv:1802.04449, Sec. IV: the
 * surface elements dSigma_mu of constant freeze-out energy density e_f, and
 * App. A.2: the surface is found between stored time slices on the device).
 *
 * Only the test suite may load this code; the HIP library shares none of it.
 *
 * The paper names the surface but not the finding algorithm (it cites earlier
 * work), so the definition used here is stated in full:
 *
 *  - Between two stored slices A (tau_A) and B (tau_B > tau_A) every group of
 *    2 x 2 x 2 x 2 grid points (two slices, two neighbouring cells per axis) is
 *    a hypercube; along an axis with a single cell the hypercube has both
 *    corners on that cell and the cell's width as its extent.
 *  - phi = e - e_f at the 16 corners.  The surface inside the hypercube is the
 *    zero set of the piecewise-linear interpolant of phi on the Kuhn
 *    triangulation (simplices ordered by a permutation of the axes).
 *  - "Hot" means phi > 0.  By the divergence theorem applied to the hot part
 *    of the hypercube, the surface covector pointing out of the hot region is
 *    S_mu = V_mu (f_lo(mu) - f_hi(mu)), where V_mu is the coordinate volume of
 *    the 3-faces normal to axis mu and f_lo / f_hi the hot volume fractions of
 *    the low / high face.  A 3-face's fraction is the mean over its six Kuhn
 *    tetrahedra of the exact hot fraction of a linear function on a
 *    tetrahedron.  Neighbouring hypercubes share their faces, so the sum of S
 *    over any set of hypercubes telescopes exactly (discrete Gauss theorem).
 *  - dSigma_mu = sqrt(-g) S_mu with sqrt(-g) = tau at the element's centre
 *    (1 in Cartesian mode), in the coordinates (tau, x, y, eta_s).
 *  - The element's centre is the mean of the points where phi changes sign
 *    along the hypercube's 32 edges (linear interpolation along each edge);
 *    e, u~ and pi~ there are the multilinear interpolants of the 16 corners.
 *
 * Element record (24 doubles): [0] hypercube index (i * cy + j) * cz + k,
 * [1..4] centre (tau, x, y, eta_s), [5..8] dSigma_mu, [9..11] u~ (x, y, eta),
 * [12..21] pi~ (zero when the slices carry no pi~), [22] e at the centre,
 * [23] zero.
 */
#include <math.h>
#include <string.h>

#define SURF_REC 24

#include "oracle_mut.h" /* planted-mistake switches (mutant build only) */

/* Hot volume fraction of a tetrahedron on which phi is linear with vertex
 * values v[0..3] (exact; every branch is a sum or product of positive terms). */
static double tet_hot_fraction(const double v[4]) {
    double pos[4], neg[4]; /* neg holds -phi >= 0 of the cold vertices */
    int np = 0, nn = 0;
    for (int t = 0; t < 4; ++t) {
        if (v[t] > 0.0)
            pos[np++] = v[t];
        else
            neg[nn++] = -v[t];
    }
    if (np == 0) return 0.0;
    if (np == 4) return 1.0;
    if (np == 1) {
        double a = pos[0];
        if (MUT(24)) return (a / (a + neg[0])) * (a / (a + neg[1]));
        return (a / (a + neg[0])) * (a / (a + neg[1])) * (a / (a + neg[2]));
    }
    if (np == 3) {
        double c = neg[0];
        if (c == 0.0) return 1.0;
        return 1.0 - (c / (pos[0] + c)) * (c / (pos[1] + c)) * (c / (pos[2] + c));
    }
    /* two hot (a, b), two cold (c, d): the volume of {phi > 0} is
     * [a^2 b^2 + a b (a + b)(c + d) + c d (a^2 + a b + b^2)] / [(a+c)(a+d)(b+c)(b+d)]
     * with c, d the magnitudes of the cold values */
    double a = pos[0], b = pos[1], c = neg[0], d = neg[1];
    double num = a * a * b * b + a * b * (a + b) * (c + d) +
                 (MUT(22) ? 0.0 : c * d * (a * a + a * b + b * b));
    double den = (a + c) * (a + d) * (b + c) * (b + d);
    return num / den;
}

/* Hot fraction of a 3-cube whose corner values are w[b] with b = 4 b0 + 2 b1 + b2
 * (b0, b1, b2 the bits of the cube's three axes in increasing axis order):
 * mean over the six Kuhn tetrahedra 000 -> +e_p -> +e_q -> 111. */
static double cube_hot_fraction(const double w[8]) {
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    static const int bitv[3] = {4, 2, 1};
    double s = 0.0;
    for (int p = 0; p < 6; ++p) {
        double v[4];
        int b = 0;
        v[0] = w[b];
        for (int t = 0; t < 3; ++t) {
            b |= bitv[perm[p][t]];
            v[t + 1] = w[b];
        }
        s += tet_hot_fraction(v);
    }
    return s / 6.0;
}

/* Hypercube corner index: c = 8 b_tau + 4 b_x + 2 b_y + b_eta. */
long orc_surface(int nx, int ny, int ne, double dx, double dy, double de, const double *A,
                 double tauA, const double *B, double tauB, int nf, double eps_f, int cartesian,
                 double *out, long capacity) {
    if (nx < 1 || ny < 1 || ne < 1 || !(tauB > tauA) || (nf != 4 && nf != 14)) return -1;
    const long ncell = (long)nx * ny * ne;
    const int cx = nx > 1 ? nx - 1 : 1, cy = ny > 1 ? ny - 1 : 1, cz = ne > 1 ? ne - 1 : 1;
    const double ext[4] = {tauB - tauA, dx, dy, de}; /* hypercube extents */
    long count = 0;
    for (int i = 0; i < cx; ++i)
        for (int j = 0; j < cy; ++j)
            for (int k = 0; k < cz; ++k) {
                const int ii[2] = {i, nx > 1 ? i + 1 : i};
                const int jj[2] = {j, ny > 1 ? j + 1 : j};
                const int kk[2] = {k, ne > 1 ? k + 1 : k};
                long cell[8];
                for (int b = 0; b < 8; ++b)
                    cell[b] = ((long)ii[(b >> 2) & 1] * ny + jj[(b >> 1) & 1]) * ne + kk[b & 1];
                double phi[16];
                int nhot = 0;
                for (int c = 0; c < 16; ++c) {
                    const double *S = (c & 8) ? B : A;
                    phi[c] = S[cell[c & 7]] - eps_f;
                    nhot += phi[c] > 0.0;
                }
                if (nhot == 0 || nhot == 16) continue;
                /* S_mu = V_mu (f_lo - f_hi); the face normal to axis mu keeps
                 * the other three axes in increasing order */
                double Sm[4];
                for (int mu = 0; mu < 4; ++mu) {
                    double f[2];
                    for (int side = 0; side < 2; ++side) {
                        double w[8];
                        for (int b = 0; b < 8; ++b) {
                            /* spread the 3 bits of b over the axes other than mu */
                            int c = 0, t = 0;
                            for (int ax = 0; ax < 4; ++ax) {
                                int bit;
                                if (ax == mu)
                                    bit = side;
                                else {
                                    bit = (b >> (2 - t)) & 1;
                                    ++t;
                                }
                                c |= bit << (3 - ax);
                            }
                            w[b] = phi[c];
                        }
                        f[side] = cube_hot_fraction(w);
                    }
                    double V = 1.0;
                    for (int ax = 0; ax < 4; ++ax)
                        if (ax != mu) V *= ext[ax];
                    Sm[mu] = V * (MUT(21) ? f[1] - f[0] : f[0] - f[1]);
                }
                /* centre: mean of the edge crossings, in units of the extents */
                double cen[4] = {0.0, 0.0, 0.0, 0.0};
                int ncross = 0;
                for (int c = 0; c < 16; ++c)
                    for (int ax = 0; ax < 4; ++ax) {
                        const int bitm = 1 << (3 - ax);
                        if (c & bitm) continue;
                        const int c2 = c | bitm;
                        if ((phi[c] > 0.0) == (phi[c2] > 0.0)) continue;
                        const double s = MUT(23) ? phi[c2] / (phi[c2] - phi[c])
                                                  : phi[c] / (phi[c] - phi[c2]);
                        for (int a2 = 0; a2 < 4; ++a2) {
                            const int bb = (c >> (3 - a2)) & 1;
                            cen[a2] += (a2 == ax) ? s : (double)bb;
                        }
                        ++ncross;
                    }
                for (int a2 = 0; a2 < 4; ++a2) cen[a2] /= (double)ncross;
                /* multilinear weights of the 16 corners at the centre */
                double wgt[16];
                for (int c = 0; c < 16; ++c) {
                    double wv = 1.0;
                    for (int a2 = 0; a2 < 4; ++a2) {
                        const int bb = (c >> (3 - a2)) & 1;
                        wv *= bb ? cen[a2] : 1.0 - cen[a2];
                    }
                    wgt[c] = wv;
                }
                const double tc = tauA + cen[0] * ext[0];
                const double xc = ((double)ii[0] - 0.5 * (nx - 1)) * dx + (nx > 1 ? cen[1] * dx : 0.0);
                const double yc = ((double)jj[0] - 0.5 * (ny - 1)) * dy + (ny > 1 ? cen[2] * dy : 0.0);
                const double ec = ((double)kk[0] - 0.5 * (ne - 1)) * de + (ne > 1 ? cen[3] * de : 0.0);
                const double sg = cartesian ? 1.0 : tc;
                if (count < capacity) {
                    double *r = out + count * SURF_REC;
                    memset(r, 0, sizeof(double) * SURF_REC);
                    r[0] = (double)(((long)i * cy + j) * cz + k);
                    r[1] = tc;
                    r[2] = xc;
                    r[3] = yc;
                    r[4] = ec;
                    for (int mu = 0; mu < 4; ++mu) r[5 + mu] = sg * Sm[mu];
                    for (int f = 0; f < nf; ++f) {
                        double v = 0.0;
                        for (int c = 0; c < 16; ++c) {
                            const double *S = (c & 8) ? B : A;
                            v += wgt[c] * S[(long)f * ncell + cell[c & 7]];
                        }
                        if (f == 0)
                            r[22] = v;
                        else
                            r[8 + f] = v; /* u~ at 9..11, pi~ at 12..21 */
                    }
                }
                ++count;
            }
    return count;
}

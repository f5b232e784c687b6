/*
 * FP64 CPU oracle of one chi^2 made-to-measure (M2M) step with moving-prior
 * regularization (MPR), after Morganti & Gerhard (2012).
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the package smoke check and the
 * benchmark's CPU-baseline leg load this library. It shares no source with
 * the HIP library and is not a fallback for it.
 *
 * Everything is scalar double precision, written as the definitions read:
 *   - weights: the paper's w_i with sum w = M initially (Sec. 3.2), carried
 *     as u_i = N w_i / M so that u_i = 1 at the start (flat priors,
 *     Sec. 2.2); w_i = u_i M / N.
 *   - model observables y_j = sum_i w_i K_j(z_i)          (Sec. 2.1, eq. obs);
 *     the density part is either top-hat radial mass bins or the spherical-
 *     harmonic coefficients a_lm,k with cloud-in-cell radial weights
 *     (Sec. 3.3, eq. alm)
 *   - time smoothing: the exponential kernel of eq. myts applied to a
 *     y that is constant over each step, i.e.
 *       ytilde <- ytilde + q (y - ytilde),  q = 1 - exp(-alpha dt),
 *     with ytilde = y at t = 0.
 *   - residuals Delta_j = (ytilde_j - Y_j) / sigma_j, chi^2 = sum Delta_j^2
 *                                                  (eqs. delta and chi)
 *   - force of change (eq. modFOC) for the weights u_i, with the chi^2
 *     gradient of y_j with respect to u_i, (M/N) K_j:
 *       G_i = mu dS/du_i - (M/N) sum_j K_j(z_i) Delta_j / sigma_j
 *       dS/du_i = -ln(u_i / uhat_i)       (mass-neutral entropy, eq. S+)
 *       dS/du_i = -ln(u_i / uhat_i) - 1   (weight entropy, eq. entropy)
 *     integrated over one step as u_i <- u_i exp(eps dt G_i), with K and
 *     Delta taken at the start of the step.
 *   - leapfrog (Sec. 4.1) in drift-kick-drift form in the fixed potential.
 *   - priors (Sec. 2.3.1): cells of a rectangular (E, x = L/L_c(E)) grid,
 *     uhat = mean u of the cell, assigned to every particle in the cell.
 *   - order within a step: force of change at z^k with Delta^k, push to
 *     z^{k+1}, deposit at z^{k+1}, smoothing and residuals, then (MPR, every
 *     prior_every correction steps) new priors from z^{k+1}.
 *
 * The Hernquist potential is eq. her (Sec. 3.1); the optional NFW halo is
 *   Phi = -G M200 / f(c) ln(1 + r/r_s) / r,  f(c) = ln(1+c) - c/(1+c),
 * and the optional logarithmic halo (Sec. 5, eq. log_halo)
 *   Phi_D = v0^2/2 ln(r0^2 + R^2 + z^2/q^2),  R^2 = x^2 + y^2.
 * With it the potential is axisymmetric (q != 1) and grows without bound;
 * circular orbits, and so L_c(E), are taken in the equatorial plane.
 * Optionally the stellar part is computed from the particles themselves (a
 * multipole expansion rebuilt every scf_every steps, see "self-consistent
 * potential" below); the prior cells then keep the analytic potential.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double G, M_star, a, upsilon; /* Hernquist mass is M_star * upsilon */
    double M200, c, r_s;          /* NFW; M200 = 0 means none */
    double v0, r0, q;             /* logarithmic halo (Sec. 5); v0 = 0 means none */
    /* self-consistent stellar potential (Sec. 2.1, Sec. 5): scf_nr = 0 means
     * none (the Hernquist part is used); else the multipole expansion of the
     * particles up to degree scf_lmax with node values at scf_nr radii
     * log-spaced over [scf_rmin, scf_rmax], rebuilt every scf_every steps */
    double scf_rmin, scf_rmax;
    int32_t scf_lmax, scf_nr, scf_every;
} orc_potential;

/* kin: 0 none, 1 v_z^2 moment, 2 Gauss-Hermite b_1..b_gh_nmax, 3 LOSVD;
 * dens: 0 n_r radial mass bins, 1 a_lm,k on a mesh of n_r radii, l <= l_max */
typedef struct {
    int32_t n_r;
    double r_min, r_max;
    int32_t n_R;
    double R_min, R_max;
    int32_t kin;
    int32_t gh_nmax;
    int32_t n_v;
    double v_min, v_max;
    int32_t dens, l_max;
} orc_layout;

/* entropy: 0 = mass-neutral S+ with moving priors, 1 = weight entropy;
 * smooth: 1 = thin-plate smoothing of the prior grid with GCV (Sec. 2.3.2);
 * cells: bit 0 = a second grid for particles with L_z < 0 (rotating models,
 * Sec. 5), bit 1 = energy bins linear in exp(E) (Sec. 5.2) */
typedef struct {
    double dt, eps, mu, alpha, mass;
    int32_t entropy, n_E, n_x, prior_every;
    double E_lo, E_hi;
    int32_t smooth, cells;
} orc_params;

/* cells of the prior grid: n_E n_x, twice that with the L_z split */
static int n_cells(const orc_params *P) {
    return P->n_E * P->n_x * ((P->cells & 1) ? 2 : 1);
}

/* position of E on the energy axis in bin units: (E - E_lo)/(E_hi - E_lo) n_E,
 * or (exp E - exp E_lo)/(exp E_hi - exp E_lo) n_E */
static double energy_coord(const orc_params *P, double E) {
    if (P->cells & 2) return (exp(E) - exp(P->E_lo)) / (exp(P->E_hi) - exp(P->E_lo)) * P->n_E;
    return (E - P->E_lo) / (P->E_hi - P->E_lo) * P->n_E;
}

typedef struct {
    int64_t n;
    double *x, *y, *z, *vx, *vy, *vz, *u, *uhat;
    orc_potential pot;
    orc_layout lay;
    orc_params par;
    int32_t J;
    const double *Y, *sigma, *Vp, *sp;
    double *ytilde, *yraw, *delta;
    double chi2;
    int64_t kstep;
    uint8_t *flag;   /* optional: particle came within `band` of an edge */
    double band;
    int32_t nthreads;
    double *ucell;   /* n_E n_x prior grid, kept between refreshes (empty cells keep theirs) */
    double *scf;     /* self-consistent potential: node table (scf_nr x (scf_lmax+1)^2 x 2) */
    int64_t tstep;   /* steps of any kind taken (the expansion's schedule) */
} orc_model;

#define ORC_MAXK 256  /* at most 2 x 81 density + 64 kinematic entries per particle */

/* ------------------------------------------------------------- potential */
static double nfw_fc(const orc_potential *p) {
    return log(1.0 + p->c) - p->c / (1.0 + p->c);
}

/* the spherical part (Hernquist + NFW) at radius r */
static double phi_sph(const orc_potential *p, double r) {
    double phi = -p->G * p->M_star * p->upsilon / (r + p->a);
    if (p->M200 > 0.0) {
        double k = p->G * p->M200 / nfw_fc(p);
        phi += (r > 0.0) ? -k * log1p(r / p->r_s) / r : -k / p->r_s;
    }
    return phi;
}

static double halo_phi(const orc_potential *p, double R2, double z2) {
    if (p->v0 == 0.0) return 0.0;
    return 0.5 * p->v0 * p->v0 * log(p->r0 * p->r0 + R2 + z2 / (p->q * p->q));
}

/* Phi at (x, y, z) */
double orc_phi3(const orc_potential *p, double x, double y, double z) {
    double R2 = x * x + y * y, z2 = z * z;
    return phi_sph(p, sqrt(R2 + z2)) + halo_phi(p, R2, z2);
}

/* Phi on the equatorial plane at radius r (the whole potential when it is
 * spherical) */
double orc_phi(const orc_potential *p, double r) {
    return phi_sph(p, r) + halo_phi(p, r * r, 0.0);
}

double orc_mass(const orc_potential *p, double r) {
    double m = p->M_star * p->upsilon * r * r / ((r + p->a) * (r + p->a));
    if (p->M200 > 0.0) {
        double x = r / p->r_s;
        m += p->M200 / nfw_fc(p) * (log1p(x) - x / (1.0 + x));
    }
    return m;
}

/* g = -grad Phi: -G M(<r) r_vec / r^3 of the spherical part (zero at the
 * centre by symmetry) and -v0^2 (x, y, z/q^2) / (r0^2 + R^2 + z^2/q^2) of the
 * logarithmic halo */
void orc_accel(const orc_potential *p, double x, double y, double z, double *g) {
    double r = sqrt(x * x + y * y + z * z);
    g[0] = g[1] = g[2] = 0.0;
    if (r > 0.0) {
        double s = -p->G * orc_mass(p, r) / (r * r * r);
        g[0] = s * x;
        g[1] = s * y;
        g[2] = s * z;
    }
    if (p->v0 != 0.0) {
        double q2 = p->q * p->q;
        double D = p->r0 * p->r0 + x * x + y * y + z * z / q2;
        double k = -p->v0 * p->v0 / D;
        g[0] += k * x;
        g[1] += k * y;
        g[2] += k * z / q2;
    }
}

/* squared circular speed at radius r in the equatorial plane, r dPhi/dR */
static double vc2(const orc_potential *p, double r) {
    double v = r > 0.0 ? p->G * orc_mass(p, r) / r : 0.0;
    if (p->v0 != 0.0) v += p->v0 * p->v0 * r * r / (p->r0 * p->r0 + r * r);
    return v;
}

/* energy of the circular orbit of radius r: Phi(r) + v_c^2/2 */
static double circ_energy(const orc_potential *p, double r) {
    return orc_phi(p, r) + 0.5 * vc2(p, r);
}

/* L_c(E): angular momentum of the circular orbit of energy E, by bisection
 * of circ_energy(r) = E. 0 for E <= Phi(0); +inf for E >= 0 when the
 * potential vanishes at infinity (no logarithmic halo). */
double orc_lc(const orc_potential *p, double E) {
    if (E <= orc_phi(p, 0.0)) return 0.0;
    if (p->v0 == 0.0 && E >= 0.0) return INFINITY;
    double lo = 0.0, hi = 1.0;
    while (circ_energy(p, hi) < E && hi < 1e300) hi *= 2.0;
    /* halve until the bracket is a few ulps wide (or stops shrinking) */
    for (int it = 0; it < 2000 && hi - lo > 4e-16 * hi; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (circ_energy(p, mid) < E) lo = mid; else hi = mid;
    }
    double rc = 0.5 * (lo + hi);
    return rc * sqrt(vc2(p, rc));
}

/* -------------------------------------------------------- observables */
/* observables of the density part: n_r bins, or (l_max + 1)^2 coefficients
 * at each of the n_r mesh radii */
static int32_t dens_J(const orc_layout *L) {
    return L->dens == 1 ? L->n_r * (L->l_max + 1) * (L->l_max + 1) : L->n_r;
}

int32_t orc_J(const orc_layout *L) {
    int32_t per = 0;
    if (L->kin == 1) per = 1;
    else if (L->kin == 2) per = L->gh_nmax;
    else if (L->kin == 3) per = L->n_v;
    return dens_J(L) + L->n_R * per;
}

/* log edges e_k = lo (hi/lo)^(k/n), e_0 = lo, e_n = hi */
static double log_edge(double lo, double hi, int n, int k) {
    if (k == 0) return lo;
    if (k == n) return hi;
    return lo * pow(hi / lo, (double)k / (double)n);
}

static double lin_edge(double lo, double hi, int n, int k) {
    if (k == 0) return lo;
    if (k == n) return hi;
    return lo + (hi - lo) * (double)k / (double)n;
}

/* index k with e_k <= v < e_{k+1}, or -1 outside [e_0, e_n) */
static int find_bin(const double *e, int n, double v) {
    if (!(v >= e[0]) || !(v < e[n])) return -1;
    for (int k = 0; k < n; ++k)
        if (v >= e[k] && v < e[k + 1]) return k;
    return -1;
}

/* physicists' Hermite polynomial, explicit sum:
 * H_n(x) = n! sum_{m=0}^{n/2} (-1)^m (2x)^(n-2m) / (m! (n-2m)!) */
double orc_hermite(int n, double x) {
    double s = 0.0;
    double nf = tgamma(n + 1.0);
    for (int m = 0; 2 * m <= n; ++m) {
        double term = pow(2.0 * x, n - 2 * m) / (tgamma(m + 1.0) * tgamma(n - 2 * m + 1.0));
        s += (m % 2 ? -term : term);
    }
    return nf * s;
}

/* Gauss-Hermite function u_n(nu) = (2^(n+1) pi n!)^(-1/2) H_n(nu) exp(-nu^2/2) */
double orc_gh_u(int n, double nu) {
    double norm = 1.0 / sqrt(pow(2.0, n + 1) * M_PI * tgamma(n + 1.0));
    return norm * orc_hermite(n, nu) * exp(-0.5 * nu * nu);
}

/* binomial coefficient C(n, k) */
static double binom(int n, int k) {
    return tgamma(n + 1.0) / (tgamma(k + 1.0) * tgamma(n - k + 1.0));
}

/* associated Legendre function with the Condon-Shortley phase,
 *   P_l^m(x) = (-1)^m (1 - x^2)^(m/2) d^m/dx^m P_l(x),  0 <= m <= l,
 * with the Legendre polynomial written out as
 *   P_l(x) = 2^-l sum_k (-1)^k C(l, k) C(2l - 2k, l) x^(l - 2k)
 * and differentiated term by term. */
double orc_plm(int l, int m, double x) {
    double d = 0.0;
    for (int k = 0; 2 * k <= l; ++k) {
        int p = l - 2 * k;
        if (p < m) continue;
        double c = ldexp(binom(l, k) * binom(2 * l - 2 * k, l), -l) * (k % 2 ? -1.0 : 1.0);
        d += c * tgamma(p + 1.0) / tgamma(p - m + 1.0) * pow(x, p - m);
    }
    return (m % 2 ? -1.0 : 1.0) * pow(1.0 - x * x, 0.5 * m) * d;
}

/* real orthonormal spherical harmonic of degree l and order m (-l..l) at
 * cos(theta) = ct and azimuth phi:
 *   m = 0: N_l0 P_l(ct),  m > 0: sqrt2 N_lm P_l^m(ct) cos(m phi),
 *   m < 0: sqrt2 N_l|m| P_l^|m|(ct) sin(|m| phi),
 *   N_lm = sqrt((2l + 1)/(4 pi) (l - m)!/(l + m)!) */
double orc_ylm(int l, int m, double ct, double phi) {
    int am = m < 0 ? -m : m;
    double N = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * tgamma(l - am + 1.0) / tgamma(l + am + 1.0));
    double P = orc_plm(l, am, ct);
    if (m == 0) return N * P;
    return sqrt(2.0) * N * P * (m > 0 ? cos(am * phi) : sin(am * phi));
}

/* ------------------------------------------------- self-consistent potential
 * The stellar potential computed from the particles as they move (Sec. 2.1;
 * in Sec. 5 from a spherical-harmonic decomposition of the model's light at a
 * constant mass-to-light ratio). The particles' masses are
 * m_i = upsilon w_i = upsilon u_i M / N. Poisson's equation in spherical
 * harmonics (the multipole expansion of the point masses), truncated at
 * l <= scf_lmax:
 *   Phi_*(x) = sum_lm Phi_lm(r) Y_lm(theta, phi),
 *   Phi_lm(r) = -4 pi G / (2l + 1) [r^-(l+1) A_lm(r) + r^l B_lm(r)],
 *   A_lm(r) = sum_{r_i < r} m_i r_i^l Y_lm(x_i),
 *   B_lm(r) = sum_{r_i >= r} m_i r_i^-(l+1) Y_lm(x_i).
 * It is taken exactly at the nodes rho_k (k < scf_nr, log-spaced over
 * [scf_rmin, scf_rmax]) together with its slope
 *   r dPhi_lm/dr = -4 pi G / (2l + 1) [-(l+1) r^-(l+1) A_lm + l r^l B_lm]
 * (the terms of dA/dr and dB/dr cancel). Between nodes Phi_lm is the cubic
 * Hermite interpolant of these values and slopes in s = ln r; inside rho_0 it
 * is the regular r^l (c0 + c1 r^2), beyond the last node the decaying
 * c0 r^-(l+1) + c1 r^-(l+3) (the potential of a bounded mass falls off; the
 * form is exact when no mass lies beyond the last node), each with the value
 * and slope of its end node. Particles with a non-finite radius add nothing.
 * Table entry
 * (k (scf_lmax+1)^2 + l^2 + l + m) 2 holds Phi_lm(rho_k), the next one
 * r dPhi_lm/dr there. */
static int nthreads_of(int32_t want);

static double scf_node(const orc_potential *p, int k) {
    if (k == 0) return p->scf_rmin;
    if (k == p->scf_nr - 1) return p->scf_rmax;
    return p->scf_rmin * pow(p->scf_rmax / p->scf_rmin, (double)k / (double)(p->scf_nr - 1));
}

void orc_scf_table(const orc_potential *p, int64_t n, const double *x, const double *y,
                   const double *z, const double *u, double mass, double *tab, int32_t nthreads) {
    const int L = p->scf_lmax, K = p->scf_nr, nlm = (L + 1) * (L + 1);
    /* per particle: r and m_i Y_lm(x_i) */
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *mY = (double *)malloc(sizeof(double) * (size_t)n * nlm);
    for (int64_t i = 0; i < n; ++i) {
        r[i] = sqrt(x[i] * x[i] + y[i] * y[i] + z[i] * z[i]);
        double ct = r[i] > 0.0 ? z[i] / r[i] : 1.0, ph = atan2(y[i], x[i]);
        double mi = p->upsilon * u[i] * mass / (double)n;
        for (int l = 0; l <= L; ++l)
            for (int m = -l; m <= l; ++m) mY[i * nlm + l * l + l + m] = mi * orc_ylm(l, m, ct, ph);
    }
    int T = nthreads_of(nthreads);
#ifdef _OPENMP
#pragma omp parallel for num_threads(T) schedule(static)
#endif
    for (int k = 0; k < K; ++k) {
        double rho = scf_node(p, k);
        for (int l = 0; l <= L; ++l)
            for (int m = -l; m <= l; ++m) {
                int lm = l * l + l + m;
                double A = 0.0, B = 0.0;
                for (int64_t i = 0; i < n; ++i) {
                    if (!isfinite(r[i])) continue;
                    if (r[i] < rho)
                        A += pow(r[i], l) * mY[i * nlm + lm];
                    else
                        B += pow(r[i], -(l + 1)) * mY[i * nlm + lm];
                }
                double c = -4.0 * M_PI * p->G / (2.0 * l + 1.0);
                double ra = pow(rho, -(l + 1)), rb = pow(rho, l);
                tab[(k * nlm + lm) * 2] = c * (ra * A + rb * B);
                tab[(k * nlm + lm) * 2 + 1] = c * (-(l + 1) * ra * A + l * rb * B);
            }
    }
    free(mY);
    free(r);
}

/* Phi_lm(r) and r dPhi_lm/dr at radius r from the node table */
static void scf_radial(const orc_potential *p, const double *tab, int nlm, int l, int lm, double r,
                       double *f, double *d) {
    const int K = p->scf_nr;
    const double r0 = scf_node(p, 0), r1 = scf_node(p, K - 1);
    if (r < r0) {
        double P = tab[lm * 2], D = tab[lm * 2 + 1], v = r / r0, vl = pow(v, l);
        double c = 0.5 * (D - l * P);
        *f = vl * (P + c * (v * v - 1.0));
        *d = vl * (l * P + c * ((l + 2) * v * v - l));
        return;
    }
    if (r >= r1) {
        const double *t = tab + ((K - 1) * nlm + lm) * 2;
        double P = t[0], D = t[1], v = r / r1;
        double b = -0.5 * (D + (l + 1) * P), a = P - b;
        double va = pow(v, -(l + 1)), iv2 = 1.0 / (v * v);
        *f = va * (a + b * iv2);
        *d = -va * ((l + 1) * a + (l + 3) * b * iv2);
        return;
    }
    int k = 0;
    while (k < K - 2 && scf_node(p, k + 1) <= r) ++k;
    const double *t0 = tab + (k * nlm + lm) * 2, *t1 = tab + ((k + 1) * nlm + lm) * 2;
    double s0 = log(scf_node(p, k)), h = log(scf_node(p, k + 1)) - s0;
    double t = (log(r) - s0) / h, t2 = t * t, t3 = t2 * t;
    *f = (2 * t3 - 3 * t2 + 1) * t0[0] + h * (t3 - 2 * t2 + t) * t0[1] + (-2 * t3 + 3 * t2) * t1[0] +
         h * (t3 - t2) * t1[1];
    *d = ((6 * t2 - 6 * t) * t0[0] + h * (3 * t2 - 4 * t + 1) * t0[1] + (-6 * t2 + 6 * t) * t1[0] +
          h * (3 * t2 - 2 * t) * t1[1]) / h;
}

double orc_scf_phi(const orc_potential *p, const double *tab, double x, double y, double z) {
    const int L = p->scf_lmax, nlm = (L + 1) * (L + 1);
    double r = sqrt(x * x + y * y + z * z);
    double ct = r > 0.0 ? z / r : 1.0, ph = atan2(y, x), phi = 0.0;
    for (int l = 0; l <= L; ++l)
        for (int m = -l; m <= l; ++m) {
            double f, d;
            scf_radial(p, tab, nlm, l, l * l + l + m, r, &f, &d);
            phi += f * orc_ylm(l, m, ct, ph);
        }
    return phi;
}

/* g = -grad Phi_* in spherical components: dPhi/dr, (1/r) dPhi/dtheta with
 *   dP_l^m/dtheta = (l cos(theta) P_l^m - (l + m) P_{l-1}^m) / sin(theta),
 * and (1/(r sin(theta))) dPhi/dphi. Zero at the centre (where the direction is
 * undefined); on the z axis the direction is tilted by 1e-9 rad. */
void orc_scf_accel(const orc_potential *p, const double *tab, double x, double y, double z,
                   double *g) {
    const int L = p->scf_lmax, nlm = (L + 1) * (L + 1);
    double r = sqrt(x * x + y * y + z * z);
    g[0] = g[1] = g[2] = 0.0;
    if (!(r > 0.0)) return;
    double R = sqrt(x * x + y * y);
    if (R == 0.0) {
        x = r * 1e-9;
        R = x;
    }
    double ct = z / r, st = R / r, cp = x / R, sp = y / R, ph = atan2(y, x);
    double dr = 0.0, dth = 0.0, dps = 0.0;
    for (int l = 0; l <= L; ++l)
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double f, d;
            scf_radial(p, tab, nlm, l, l * l + l + m, r, &f, &d);
            double N = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * tgamma(l - am + 1.0) /
                            tgamma(l + am + 1.0));
            double P = orc_plm(l, am, ct);
            double Pm1 = (l - 1 >= am) ? orc_plm(l - 1, am, ct) : 0.0;
            double dP = (l * ct * P - (l + am) * Pm1) / st;
            double T, dT; /* the azimuthal factor and its phi derivative */
            if (m == 0) {
                T = 1.0;
                dT = 0.0;
            } else if (m > 0) {
                T = sqrt(2.0) * cos(am * ph);
                dT = -sqrt(2.0) * am * sin(am * ph);
            } else {
                T = sqrt(2.0) * sin(am * ph);
                dT = sqrt(2.0) * am * cos(am * ph);
            }
            dr += d / r * N * P * T;
            dth += f * N * dP * T;
            dps += f * N * P / st * dT;
        }
    /* grad = dr rhat + dth/r thetahat + dps/r phihat */
    double gt = dth / r, gp = dps / r;
    g[0] = -(dr * st * cp + gt * ct * cp - gp * sp);
    g[1] = -(dr * st * sp + gt * ct * sp + gp * cp);
    g[2] = -(dr * ct - gt * st);
}

typedef struct {
    int32_t nr, nR, nv;
    double *re, *Re, *ve;
} edges_t;

/* density edges: n_r + 1 bin edges, or the n_r mesh radii (n_r - 1 intervals),
 * both log-spaced from r_min to r_max */
static void edges_make(const orc_layout *L, edges_t *E) {
    E->nr = L->dens == 1 ? L->n_r - 1 : L->n_r;
    E->nR = L->n_R;
    E->nv = (L->kin == 3) ? L->n_v : 0;
    E->re = (double *)malloc(sizeof(double) * (E->nr + 1));
    E->Re = (double *)malloc(sizeof(double) * (E->nR + 1));
    E->ve = (double *)malloc(sizeof(double) * (E->nv + 1));
    for (int k = 0; k <= E->nr; ++k) E->re[k] = log_edge(L->r_min, L->r_max, E->nr, k);  /* mesh r_k */
    for (int k = 0; k <= E->nR; ++k) E->Re[k] = log_edge(L->R_min, L->R_max, E->nR, k);
    for (int k = 0; k <= E->nv; ++k) E->ve[k] = lin_edge(L->v_min, L->v_max, E->nv, k);
}

static void edges_free(edges_t *E) {
    free(E->re);
    free(E->Re);
    free(E->ve);
}

static int near_edge(const double *e, int n, double v, double band, int absolute) {
    for (int k = 0; k <= n; ++k) {
        double tol = absolute ? band * fmax(1.0, fabs(e[k])) : band * e[k];
        if (fabs(v - e[k]) <= tol) return 1;
    }
    return 0;
}

/* The kernels K_j(z) that are non-zero for one phase-space point: writes
 * (index, value) pairs and returns their count. Observable order: first the
 * density part, then per annulus p (R = sqrt(x^2+y^2), line of sight z) its
 * kinematic entries: v_z^2 (kin 1), 2 sqrt(pi) u_n(nu), nu = (v_z - V_p)/sigma_p,
 * n = 1..gh_nmax (kin 2, eq. lumghn), or K = 1 for the LOSVD bin holding v_z
 * (kin 3). The density part is n_r radial mass bins (K = 1 for r in the bin,
 * dens 0) or the coefficients a_lm,k (dens 1, eq. alm): entry
 * k (l_max + 1)^2 + l^2 + l + m holds gamma_k(r) Y_l^m(theta, phi), where
 * gamma_k is the cloud-in-cell weight of mesh radius r_k, linear in r between
 * the two mesh radii around r (r_k <= r < r_{k+1}: gamma_k = (r_{k+1} - r) /
 * (r_{k+1} - r_k), gamma_{k+1} = 1 - gamma_k). A particle outside every range
 * has no kernel (selection function, Sec. 2.1). */
static int kernels(const orc_layout *L, const edges_t *E, const double *Vp, const double *sp,
                   double x, double y, double z, double vz, int *idx, double *val) {
    int cnt = 0;
    double r = sqrt(x * x + y * y + z * z);
    int k = find_bin(E->re, E->nr, r);
    if (k >= 0 && L->dens == 1) {
        int nlm = (L->l_max + 1) * (L->l_max + 1);
        double g = (E->re[k + 1] - r) / (E->re[k + 1] - E->re[k]);
        double ct = z / r, phi = atan2(y, x);
        for (int l = 0; l <= L->l_max; ++l)
            for (int m = -l; m <= l; ++m) {
                double Y = orc_ylm(l, m, ct, phi);
                idx[cnt] = k * nlm + l * l + l + m;
                val[cnt++] = g * Y;
                idx[cnt] = (k + 1) * nlm + l * l + l + m;
                val[cnt++] = (1.0 - g) * Y;
            }
    } else if (k >= 0) {
        idx[cnt] = k;
        val[cnt++] = 1.0;
    }
    if (L->kin == 0 || L->n_R == 0) return cnt;
    double R = sqrt(x * x + y * y);
    int p = find_bin(E->Re, E->nR, R);
    if (p < 0) return cnt;
    int j0 = dens_J(L);
    if (L->kin == 1) {
        idx[cnt] = j0 + p;
        val[cnt++] = vz * vz;
    } else if (L->kin == 2) {
        double nu = (vz - Vp[p]) / sp[p];
        for (int n = 1; n <= L->gh_nmax; ++n) {
            idx[cnt] = j0 + p * L->gh_nmax + (n - 1);
            val[cnt++] = 2.0 * sqrt(M_PI) * orc_gh_u(n, nu);
        }
    } else if (L->kin == 3) {
        int b = find_bin(E->ve, E->nv, vz);
        if (b >= 0) {
            idx[cnt] = j0 + p * L->n_v + b;
            val[cnt++] = 1.0;
        }
    }
    return cnt;
}

/* exported single-point evaluation (tests) */
int orc_kernels(const orc_layout *L, const double *Vp, const double *sp, double x, double y,
                double z, double vz, int32_t *idx, double *val) {
    edges_t E;
    edges_make(L, &E);
    int ii[ORC_MAXK];
    int n = kernels(L, &E, Vp, sp, x, y, z, vz, ii, val);
    for (int k = 0; k < n; ++k) idx[k] = ii[k];
    edges_free(&E);
    return n;
}

/* within `band` of an edge where a kernel jumps: every bin edge, or only
 * the two ends of the a_lm mesh (the cloud-in-cell weights are continuous
 * inside it) */
static int particle_ambiguous(const orc_layout *L, const edges_t *E, double x, double y,
                              double z, double vz, double band) {
    double r = sqrt(x * x + y * y + z * z);
    if (L->dens == 1) {
        double ends[2] = {E->re[0], E->re[E->nr]};
        if (near_edge(ends, 1, r, band, 0)) return 1;
    } else if (near_edge(E->re, E->nr, r, band, 0)) {
        return 1;
    }
    if (L->kin == 0 || L->n_R == 0) return 0;
    double R = sqrt(x * x + y * y);
    if (near_edge(E->Re, E->nR, R, band, 0)) return 1;
    if (L->kin == 3 && near_edge(E->ve, E->nv, vz, band, 1)) return 1;
    return 0;
}

static int nthreads_of(int32_t want) {
#ifdef _OPENMP
    return want > 0 ? want : 1;
#else
    (void)want;
    return 1;
#endif
}

/* y_j = (M/N) sum_i u_i K_j(z_i). Optional: yabs_j = (M/N) sum |u_i K_ij|,
 * yamb_j = the same sum over particles within `band` of an edge. With
 * several threads each thread sums its contiguous block of particles and the
 * blocks are added in thread order. */
void orc_deposit(int64_t n, const double *x, const double *y, const double *z, const double *vx,
                 const double *vy, const double *vz, const double *u, int64_t n_norm, double mass,
                 const orc_layout *L, const double *Vp, const double *sp, double *yout,
                 double *yabs, double *yamb, double band, int32_t nthreads) {
    (void)vx;
    (void)vy;
    int J = orc_J(L);
    edges_t E;
    edges_make(L, &E);
    int T = nthreads_of(nthreads);
    double *acc = (double *)calloc((size_t)T * J * 3, sizeof(double));
    double w0 = mass / (double)n_norm;
#ifdef _OPENMP
#pragma omp parallel num_threads(T)
#endif
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        int64_t lo = n * t / T, hi = n * (t + 1) / T;
        double *a = acc + (size_t)t * J * 3;
        int idx[ORC_MAXK];
        double val[ORC_MAXK];
        for (int64_t i = lo; i < hi; ++i) {
            int m = kernels(L, &E, Vp, sp, x[i], y[i], z[i], vz[i], idx, val);
            for (int k = 0; k < m; ++k) {
                double wk = w0 * u[i] * val[k];
                a[idx[k]] += wk;
                a[J + idx[k]] += fabs(wk);
            }
            if (yamb && particle_ambiguous(L, &E, x[i], y[i], z[i], vz[i], band)) {
                /* a point this close to an edge may fall on either side of it:
                 * its |w K| counts as ambiguous for every bin it reaches when r,
                 * R or v_z moves by twice the band either way */
                const double f[7][4] = {{1, 1, 1, 0},         {1 + 2 * band, 1 + 2 * band, 1 + 2 * band, 0},
                                        {1 - 2 * band, 1 - 2 * band, 1 - 2 * band, 0},
                                        {1 + 2 * band, 1 + 2 * band, 1, 0},
                                        {1 - 2 * band, 1 - 2 * band, 1, 0},
                                        {1, 1, 1, 2 * band},  {1, 1, 1, -2 * band}};
                double seen[ORC_MAXK * 7];
                int nseen = 0;
                for (int v = 0; v < 7; ++v) {
                    double dv = f[v][3] * fmax(1.0, fabs(vz[i]));
                    int mm = kernels(L, &E, Vp, sp, x[i] * f[v][0], y[i] * f[v][1], z[i] * f[v][2],
                                     vz[i] + dv, idx, val);
                    for (int k = 0; k < mm; ++k) {
                        int dup = 0;
                        for (int q = 0; q < nseen; ++q) dup |= (seen[q] == (double)idx[k]);
                        if (dup) continue;
                        seen[nseen++] = (double)idx[k];
                        a[2 * J + idx[k]] += fabs(w0 * u[i] * val[k]);
                    }
                }
            }
        }
    }
    for (int j = 0; j < J; ++j) {
        double s = 0.0, sa = 0.0, sb = 0.0;
        for (int t = 0; t < T; ++t) {
            s += acc[(size_t)t * J * 3 + j];
            sa += acc[(size_t)t * J * 3 + J + j];
            sb += acc[(size_t)t * J * 3 + 2 * J + j];
        }
        yout[j] = s;
        if (yabs) yabs[j] = sa;
        if (yamb) yamb[j] = sb;
    }
    free(acc);
    edges_free(&E);
}

/* ------------------------------------------------------------ MPR cells */
/* E = v^2/2 + Phi(r), L = |r x v|, x = L / L_c(E). Cell (k, l) of the
 * rectangular grid: k from E on [E_lo, E_hi) in n_E equal bins, l from x on
 * [0, 1) in n_x equal bins; out-of-range values go to the end cells. For
 * E >= 0 there is no circular orbit and x is taken as 0; for E <= Phi(0)
 * L_c = 0 and x is taken as 1. Returns k * n_x + l. */
/* cell of a phase-space point; also E, x and L_z / (|r| |v|) */
static int32_t cell_of(const orc_potential *p, const orc_params *P, double x, double y, double z,
                       double vx, double vy, double vz, double *Eout, double *xout,
                       double *lzout) {
    double r = sqrt(x * x + y * y + z * z);
    double E = 0.5 * (vx * vx + vy * vy + vz * vz) + orc_phi3(p, x, y, z);
    double lx = y * vz - z * vy, ly = z * vx - x * vz, lz = x * vy - y * vx;
    double L = sqrt(lx * lx + ly * ly + lz * lz);
    double xc;
    if (p->v0 == 0.0 && E >= 0.0) xc = 0.0;
    else {
        double Lc = orc_lc(p, E);
        xc = (Lc > 0.0) ? L / Lc : 1.0;
    }
    int k = (int)floor(energy_coord(P, E));
    if (!(E - P->E_lo >= 0.0)) k = 0;
    if (k < 0) k = 0;
    if (k > P->n_E - 1) k = P->n_E - 1;
    int l = (int)floor(xc * P->n_x);
    if (l < 0) l = 0;
    if (l > P->n_x - 1) l = P->n_x - 1;
    if (Eout) *Eout = E;
    if (xout) *xout = xc;
    if (lzout) {
        double rv = r * sqrt(vx * vx + vy * vy + vz * vz);
        *lzout = rv > 0.0 ? lz / rv : 0.0;
    }
    int c = k * P->n_x + l;
    if ((P->cells & 1) && lz < 0.0) c += P->n_E * P->n_x;
    return c;
}

int32_t orc_cell(const orc_potential *p, const orc_params *P, double x, double y, double z,
                 double vx, double vy, double vz, double *Eout, double *xout) {
    return cell_of(p, P, x, y, z, vx, vy, vz, Eout, xout, NULL);
}

static int cell_ambiguous(const orc_params *P, double E, double xc, double lzr, double band) {
    /* bin width in E at E: 1 / (d energy_coord / dE) */
    double dE = (P->E_hi - P->E_lo) / P->n_E;
    if (P->cells & 2) dE = (exp(P->E_hi) - exp(P->E_lo)) / (P->n_E * exp(E));
    double t = energy_coord(P, E);
    double fe = t - floor(t);
    if ((fe * dE <= band * fabs(P->E_lo) || (1.0 - fe) * dE <= band * fabs(P->E_lo)) &&
        t > 0.5 && t < P->n_E - 0.5)
        return 1;
    if ((P->cells & 1) && fabs(lzr) <= band) return 1;
    double tx = xc * P->n_x;
    double fx = tx - floor(tx);
    if ((fx <= band * P->n_x || 1.0 - fx <= band * P->n_x) && tx > 0.5 && tx < P->n_x - 0.5)
        return 1;
    return 0;
}

/* per-particle cells (tests and diagnostics) */
void orc_cells(const orc_potential *p, const orc_params *P, int64_t n, const double *x,
               const double *y, const double *z, const double *vx, const double *vy,
               const double *vz, int32_t *cell, double *E, double *xc) {
    for (int64_t i = 0; i < n; ++i)
        cell[i] = orc_cell(p, P, x[i], y[i], z[i], vx[i], vy[i], vz[i], E ? E + i : NULL,
                           xc ? xc + i : NULL);
}

/* ----------------------------------------------------------------- model */
static void residuals(orc_model *m) {
    double c2 = 0.0;
    for (int j = 0; j < m->J; ++j) {
        m->delta[j] = (m->ytilde[j] - m->Y[j]) / m->sigma[j];
        c2 += m->delta[j] * m->delta[j];
    }
    m->chi2 = c2;
}

static void deposit_model(orc_model *m, double *out) {
    orc_deposit(m->n, m->x, m->y, m->z, m->vx, m->vy, m->vz, m->u, m->n, m->par.mass, &m->lay,
                m->Vp, m->sp, out, NULL, NULL, 0.0, m->nthreads);
}

/* t = 0: ytilde = y^0 = deposit of the initial state, then Delta, chi^2 */
int orc_init(orc_model *m) {
    if (m->J != orc_J(&m->lay)) return 1;
    deposit_model(m, m->yraw);
    for (int j = 0; j < m->J; ++j) m->ytilde[j] = m->yraw[j];
    residuals(m);
    if (m->pot.scf_nr > 0) {
        if (!m->scf) return 1;
        orc_scf_table(&m->pot, m->n, m->x, m->y, m->z, m->u, m->par.mass, m->scf, m->nthreads);
    }
    return 0;
}

/* the whole acceleration of the fit: with the self-consistent potential the
 * expansion replaces the Hernquist part */
static void accel_total(const orc_model *m, double x, double y, double z, double *g) {
    if (m->pot.scf_nr == 0) {
        orc_accel(&m->pot, x, y, z, g);
        return;
    }
    orc_potential d = m->pot;
    d.M_star = 0.0;
    orc_accel(&d, x, y, z, g);
    double gs[3];
    orc_scf_accel(&m->pot, m->scf, x, y, z, gs);
    g[0] += gs[0];
    g[1] += gs[1];
    g[2] += gs[2];
}

/* ------------------------------------------------------------- smoothing
 * Thin-plate smoothing of the prior grid (Sec. 2.3.2, eq. smooth_grid), written
 * out as its definition: the smoothed grid w minimizes
 *   sum_c (w_c - w0_c)^2 + lambda w^T P w,
 * where w^T P w is the sum over the grid of the finite-difference thin-plate
 * terms (d2w/dE2)^2 + 2 (d2w/dEdx)^2 + (d2w/dx2)^2 in the grid's own units
 * (cell widths hE = (E_hi - E_lo)/n_E, or (exp E_hi - exp E_lo)/n_E for
 * energy bins linear in exp(E), and hx = 1/n_x). Each derivative is a
 * finite difference taken only where its stencil lies inside the grid, with
 * no values invented beyond an edge:
 *   d2w/dE2 at every cell with a neighbour on both sides along E,
 *     (w[k+1][l] - 2 w[k][l] + w[k-1][l]) / hE^2;
 *   d2w/dx2 likewise along x;
 *   d2w/dEdx at every interior corner of four cells,
 *     (w[k+1][l+1] - w[k+1][l] - w[k][l+1] + w[k][l]) / (hE hx).
 * Every term vanishes on a plane a + b E + c x, so lambda -> infinity gives
 * the least-squares plane, and lambda -> 0 the data. P is the sum of d d^T
 * over those stencils d; w = (I + lambda P)^-1 w0, solved here densely
 * (Cholesky). lambda minimizes the generalized cross validation score
 *   GCV(lambda) = (|w0 - A w0|^2 / n) / (1 - tr(A)/n)^2,  A = (I + lambda P)^-1,
 * searched over p = log10(lambda) in three stages: steps of 0.25 over
 * [p_lo, p_hi], then 65 points over the two steps around the best point,
 * then 65 points over the two sub-steps around the best one (first minimum
 * on ties). p_lo = -2 log10(G_hi) - 4, p_hi = -2 log10(G_lo) + 4 with G_hi =
 * 4/hE^2 + 4/hx^2 and G_lo the smaller of 4 sin^2(pi/(2n))/h^2 over the axes
 * with more than one cell (bounds of the spectrum of P from the grid
 * Laplacian, widened by four decades). The smoothed priors are floored at
 * 1e-3 times the mean of w0 (a prior must stay positive). Dense: meant for
 * small grids. */
static int cholesky(double *A, int n) {  /* in place, lower triangle */
    for (int j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
        if (!(d > 0)) return 1;
        d = sqrt(d);
        A[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double v = A[i * n + j];
            for (int k = 0; k < j; ++k) v -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = v / d;
        }
    }
    return 0;
}

/* GCV score of lambda; the smoothed grid into w if w != NULL */
static double gcv_dense(const double *P, const double *w0, int n, double lam, double *w,
                        double *scratch /* 2 n^2 + n */) {
    double *M = scratch, *Li = scratch + (size_t)n * n, *s = scratch + 2 * (size_t)n * n;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) M[i * n + j] = (i == j ? 1.0 : 0.0) + lam * P[i * n + j];
    if (cholesky(M, n)) return INFINITY;
    /* solve L L^T s = w0 */
    for (int i = 0; i < n; ++i) {
        double v = w0[i];
        for (int k = 0; k < i; ++k) v -= M[i * n + k] * s[k];
        s[i] = v / M[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double v = s[i];
        for (int k = i + 1; k < n; ++k) v -= M[k * n + i] * s[k];
        s[i] = v / M[i * n + i];
    }
    /* tr(A) = tr(L^-T L^-1) = sum of squares of the entries of L^-1 */
    double tr = 0.0;
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < j; ++i) Li[i * n + j] = 0.0;
        for (int i = j; i < n; ++i) {
            double v = (i == j) ? 1.0 : 0.0;
            for (int k = j; k < i; ++k) v -= M[i * n + k] * Li[k * n + j];
            Li[i * n + j] = v / M[i * n + i];
            tr += Li[i * n + j] * Li[i * n + j];
        }
    }
    double rss = 0.0;
    for (int i = 0; i < n; ++i) rss += (w0[i] - s[i]) * (w0[i] - s[i]);
    if (w)
        for (int i = 0; i < n; ++i) w[i] = s[i];
    double den = 1.0 - tr / n;
    return (rss / n) / (den * den);
}

/* smooth the n_E x n_x grid w (cell k n_x + l) in place; *lambda_out the
 * chosen lambda (0 if the grid has one cell) */
/* lambda_in > 0: smooth with that lambda instead of searching for it */
static int smooth_grid(const orc_params *par, double *w, double lambda_in, double *lambda_out) {
    const int nE = par->n_E, nx = par->n_x, n = nE * nx;
    if (lambda_out) *lambda_out = 0.0;
    if (n < 2) return 0;
    /* cell width along the energy axis, in the variable the bins are linear in */
    const double hE = (par->cells & 2) ? (exp(par->E_hi) - exp(par->E_lo)) / nE
                                        : (par->E_hi - par->E_lo) / nE;
    const double hx = 1.0 / nx;
    double *P = (double *)calloc((size_t)n * n, sizeof(double));
    double *w0 = (double *)malloc(sizeof(double) * n);
    double *scratch = (double *)malloc(sizeof(double) * (2 * (size_t)n * n + n));
    if (!P || !w0 || !scratch) return 1;
    for (int c = 0; c < n; ++c) w0[c] = w[c];
    /* P = sum over the stencils of weight * d d^T; a stencil d is given by
     * up to four (cell, coefficient) pairs */
    int sc[4];
    double sv[4];
#define ADD_STENCIL(cnt, weight)                                              \
    for (int a_ = 0; a_ < (cnt); ++a_)                                        \
        for (int b_ = 0; b_ < (cnt); ++b_)                                    \
            P[(size_t)sc[a_] * n + sc[b_]] += (weight) * sv[a_] * sv[b_];
    for (int k = 1; k + 1 < nE; ++k) /* d2w/dE2 */
        for (int l = 0; l < nx; ++l) {
            sc[0] = (k - 1) * nx + l; sv[0] = 1.0 / (hE * hE);
            sc[1] = k * nx + l;       sv[1] = -2.0 / (hE * hE);
            sc[2] = (k + 1) * nx + l; sv[2] = 1.0 / (hE * hE);
            ADD_STENCIL(3, 1.0)
        }
    for (int k = 0; k < nE; ++k) /* d2w/dx2 */
        for (int l = 1; l + 1 < nx; ++l) {
            sc[0] = k * nx + l - 1; sv[0] = 1.0 / (hx * hx);
            sc[1] = k * nx + l;     sv[1] = -2.0 / (hx * hx);
            sc[2] = k * nx + l + 1; sv[2] = 1.0 / (hx * hx);
            ADD_STENCIL(3, 1.0)
        }
    for (int k = 0; k + 1 < nE; ++k) /* d2w/dEdx, counted twice */
        for (int l = 0; l + 1 < nx; ++l) {
            sc[0] = (k + 1) * nx + l + 1; sv[0] = 1.0 / (hE * hx);
            sc[1] = (k + 1) * nx + l;     sv[1] = -1.0 / (hE * hx);
            sc[2] = k * nx + l + 1;       sv[2] = -1.0 / (hE * hx);
            sc[3] = k * nx + l;           sv[3] = 1.0 / (hE * hx);
            ADD_STENCIL(4, 2.0)
        }
#undef ADD_STENCIL
    /* search range */
    double Ghi = 0.0, Glo = INFINITY;
    if (nE > 1) {
        Ghi += 4.0 / (hE * hE);
        const double s = sin(M_PI / (2.0 * nE));
        Glo = fmin(Glo, 4.0 * s * s / (hE * hE));
    }
    if (nx > 1) {
        Ghi += 4.0 / (hx * hx);
        const double s = sin(M_PI / (2.0 * nx));
        Glo = fmin(Glo, 4.0 * s * s / (hx * hx));
    }
    const double plo = -2.0 * log10(Ghi) - 4.0, phi_ = -2.0 * log10(Glo) + 4.0;
    const int K1 = lambda_in > 0.0 ? 0 : (int)floor((phi_ - plo) / 0.25) + 1;
    int best = 0;
    double bg = INFINITY;
    for (int i = 0; i < K1; ++i) {
        const double g = gcv_dense(P, w0, n, pow(10.0, plo + 0.25 * i), NULL, scratch);
        if (g < bg) { bg = g; best = i; }
    }
    double a = plo + 0.25 * (best > 0 ? best - 1 : 0);
    double b = plo + 0.25 * (best < K1 - 1 ? best + 1 : K1 - 1);
    for (int stage = 0; stage < 2 && K1 > 0; ++stage) {
        int bi = 0;
        bg = INFINITY;
        for (int j = 0; j <= 64; ++j) {
            const double g = gcv_dense(P, w0, n, pow(10.0, a + (b - a) * j / 64.0), NULL, scratch);
            if (g < bg) { bg = g; bi = j; }
        }
        const double na = a + (b - a) * (bi > 0 ? bi - 1 : 0) / 64.0;
        const double nb = a + (b - a) * (bi < 64 ? bi + 1 : 64) / 64.0;
        if (stage == 1) { a = a + (b - a) * bi / 64.0; b = a; break; }
        a = na;
        b = nb;
    }
    const double lam = lambda_in > 0.0 ? lambda_in : pow(10.0, a);
    (void)gcv_dense(P, w0, n, lam, w, scratch);
    double mean = 0.0;
    for (int c = 0; c < n; ++c) mean += w0[c];
    mean /= n;
    for (int c = 0; c < n; ++c) w[c] = fmax(w[c], 1e-3 * mean);
    if (lambda_out) *lambda_out = lam;
    free(P);
    free(w0);
    free(scratch);
    return 0;
}

int orc_smooth_grid(const orc_params *par, double *w, double *lambda_out) {
    return smooth_grid(par, w, 0.0, lambda_out);
}

/* the smoothed grid at a given lambda > 0 (tests of the lambda search) */
int orc_smooth_grid_at(const orc_params *par, double *w, double lambda) {
    return smooth_grid(par, w, lambda > 0.0 ? lambda : 1e-300, NULL);
}

/* new priors: uhat_i = prior of the (E, x) cell of particle i, the mean of u
 * over the cell (empty cells keep their previous prior), then optionally
 * smoothed over the grid */
int orc_refresh_priors(orc_model *m) {
    int C = n_cells(&m->par);
    double *sum = (double *)calloc(C, sizeof(double));
    int64_t *cnt = (int64_t *)calloc(C, sizeof(int64_t));
    int32_t *cell = (int32_t *)malloc(sizeof(int32_t) * m->n);
    int T = nthreads_of(m->nthreads);
#ifdef _OPENMP
#pragma omp parallel for num_threads(T) schedule(static)
#endif
    for (int64_t i = 0; i < m->n; ++i) {
        double E, xc, lzr;
        cell[i] = cell_of(&m->pot, &m->par, m->x[i], m->y[i], m->z[i], m->vx[i], m->vy[i],
                          m->vz[i], &E, &xc, &lzr);
        if (m->flag && cell_ambiguous(&m->par, E, xc, lzr, m->band)) m->flag[i] = 1;
    }
    /* cell sums in particle order */
    for (int64_t i = 0; i < m->n; ++i) {
        sum[cell[i]] += m->u[i];
        cnt[cell[i]] += 1;
    }
    double *grid = (double *)malloc(sizeof(double) * C);
    for (int c = 0; c < C; ++c)
        grid[c] = cnt[c] > 0 ? sum[c] / (double)cnt[c] : (m->ucell ? m->ucell[c] : 1.0);
    int rc = 0;
    /* each n_E x n_x grid (both halves with the L_z split) is smoothed alone */
    if (m->par.smooth)
        for (int c0 = 0; c0 < C && rc == 0; c0 += m->par.n_E * m->par.n_x)
            rc = orc_smooth_grid(&m->par, grid + c0, NULL);
    if (m->ucell)
        for (int c = 0; c < C; ++c) m->ucell[c] = grid[c];
    for (int64_t i = 0; i < m->n; ++i) m->uhat[i] = grid[cell[i]];
    free(grid);
    free(sum);
    free(cnt);
    free(cell);
    return rc;
}

/* One drift-kick-drift leapfrog step (Sec. 4.1) of one particle: drift half
 * a step, kick a whole step with the acceleration at the midpoint, drift half
 * a step. The acceleration comes from acc(ctx, x, y, z, g). Both the step loop
 * of a fit and the bare integrator below use this one function. */
typedef void (*orc_accel_fn)(const void *ctx, double x, double y, double z, double *g);

static void dkd_step(double dt, double *x, double *y, double *z, double *vx, double *vy,
                     double *vz, orc_accel_fn acc, const void *ctx) {
    double g[3];
    *x += 0.5 * dt * *vx;
    *y += 0.5 * dt * *vy;
    *z += 0.5 * dt * *vz;
    acc(ctx, *x, *y, *z, g);
    *vx += dt * g[0];
    *vy += dt * g[1];
    *vz += dt * g[2];
    *x += 0.5 * dt * *vx;
    *y += 0.5 * dt * *vy;
    *z += 0.5 * dt * *vz;
}

/* the acceleration of a fit (analytic, or with its self-consistent part) */
static void accel_of_model(const void *ctx, double x, double y, double z, double *g) {
    accel_total((const orc_model *)ctx, x, y, z, g);
}

/* the acceleration of a fixed analytic potential */
static void accel_of_potential(const void *ctx, double x, double y, double z, double *g) {
    orc_accel((const orc_potential *)ctx, x, y, z, g);
}

/* n steps; correct = 0 advances and smooths without weight correction
 * (relaxation). chi2_hist (optional) receives chi^2 after each step. */
int orc_steps(orc_model *m, int32_t nsteps, int32_t correct, double *chi2_hist) {
    const orc_params *P = &m->par;
    double dt = P->dt;
    double q = -expm1(-P->alpha * dt);
    double cS = (P->entropy == 1) ? 1.0 : 0.0;
    double w0 = P->mass / (double)m->n;
    edges_t E;
    edges_make(&m->lay, &E);
    double *rj = (double *)malloc(sizeof(double) * m->J);
    int T = nthreads_of(m->nthreads);
    for (int s = 0; s < nsteps; ++s) {
        for (int j = 0; j < m->J; ++j) rj[j] = m->delta[j] / m->sigma[j];
#ifdef _OPENMP
#pragma omp parallel for num_threads(T) schedule(static)
#endif
        for (int64_t i = 0; i < m->n; ++i) {
            int idx[ORC_MAXK];
            double val[ORC_MAXK];
            if (correct) {
                /* force of change at z^k with Delta^k */
                int cnt = kernels(&m->lay, &E, m->Vp, m->sp, m->x[i], m->y[i], m->z[i], m->vz[i],
                                  idx, val);
                double chi = 0.0;
                for (int k = 0; k < cnt; ++k) chi += val[k] * rj[idx[k]];
                double G = P->mu * (-log(m->u[i] / m->uhat[i]) - cS) - w0 * chi;
                m->u[i] *= exp(P->eps * dt * G);
            }
            dkd_step(dt, &m->x[i], &m->y[i], &m->z[i], &m->vx[i], &m->vy[i], &m->vz[i],
                     accel_of_model, m);
            if (m->flag &&
                particle_ambiguous(&m->lay, &E, m->x[i], m->y[i], m->z[i], m->vz[i], m->band))
                m->flag[i] = 1;
        }
        deposit_model(m, m->yraw);
        for (int j = 0; j < m->J; ++j) m->ytilde[j] += q * (m->yraw[j] - m->ytilde[j]);
        residuals(m);
        if (correct) {
            m->kstep += 1;
            if (P->entropy == 0 && P->prior_every > 0 && m->kstep % P->prior_every == 0)
                orc_refresh_priors(m);
        }
        /* the self-consistent potential from z^{k+1} and the new weights */
        m->tstep += 1;
        if (m->pot.scf_nr > 0 && m->tstep % m->pot.scf_every == 0)
            orc_scf_table(&m->pot, m->n, m->x, m->y, m->z, m->u, P->mass, m->scf, m->nthreads);
        if (chi2_hist) chi2_hist[s] = m->chi2;
    }
    free(rj);
    edges_free(&E);
    return 0;
}

/* sum of w = u M / N per (E, x) cell (the grid diagnostic of Sec. 4.1) */
void orc_cell_mass(const orc_potential *p, const orc_params *P, int64_t n, const double *x,
                   const double *y, const double *z, const double *vx, const double *vy,
                   const double *vz, const double *u, double mass, double *out) {
    int C = n_cells(P);
    for (int c = 0; c < C; ++c) out[c] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        int32_t c = orc_cell(p, P, x[i], y[i], z[i], vx[i], vy[i], vz[i], NULL, NULL);
        out[c] += u[i] * mass / (double)n;
    }
}

/* nsteps DKD steps of n particles in a fixed potential (tests of the
 * integrator): the same step function as the fit's step loop */
void orc_push(const orc_potential *p, double dt, int64_t n, double *x, double *y, double *z,
              double *vx, double *vy, double *vz, int32_t nsteps) {
    for (int s = 0; s < nsteps; ++s)
        for (int64_t i = 0; i < n; ++i)
            dkd_step(dt, &x[i], &y[i], &z[i], &vx[i], &vy[i], &vz[i], accel_of_potential, p);
}

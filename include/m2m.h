/*
 * m2m.h -- C ABI of the made-to-measure (chi^2 M2M) step with moving-prior
 * regularization on AMD Instinct MI355X (gfx950).
 *
 * The operations follow Morganti & Gerhard (2012), "Regularizing
 * made-to-measure particle models of galaxies":
 *   - particles z_i = (r_i, v_i) with weights w_i orbit in a fixed potential
 *     (Sec. 2.1); they advance by a drift-kick-drift leapfrog (Sec. 4.1);
 *   - model observables y_j = sum_i w_i K_j(z_i) (Sec. 2.1, eq. obs) with a
 *     selection function, time-smoothed by the exponential kernel of eq. myts;
 *   - residuals Delta_j = (ytilde_j - Y_j) / sigma(Y_j) and
 *     chi^2 = sum_j Delta_j^2 (eqs. delta, chi);
 *   - force of change (eq. modFOC) with the mass-neutral entropy S+ (eq. S+)
 *     or the weight entropy (eq. entropy);
 *   - moving priors (Sec. 2.3.1): mean weight in cells of an (E, x = L/L_c)
 *     grid assigned as the prior of every particle in the cell;
 *   - optionally: thin-plate smoothing of the prior grid (Sec. 2.3.2), the
 *     spherical-harmonic density observables a_lm (Sec. 3.3), prior cells for
 *     rotating models and a logarithmic halo (Sec. 5), and the stellar
 *     potential computed from the particles themselves (Sec. 2.1, Sec. 5).
 *
 * Conventions fixed by this interface
 *   Weights. The library carries u_i = N w_i / M ("u", 1 for equal weights;
 *     M = params.mass) and the priors uhat_i in the same units. The model
 *     observable is y_j = (M/N) sum_i u_i K_j(z_i). The force of change per
 *     step of length dt, with K and Delta taken at the start of the step, is
 *       u_i <- u_i exp(eps dt G_i),
 *       G_i = mu dS/du_i - (M/N) sum_j K_j(z_i) Delta_j / sigma_j,
 *       dS/du_i = -ln(u_i/uhat_i)        (M2M_S_MPR, eq. S+)
 *       dS/du_i = -ln(u_i/uhat_i) - 1    (M2M_S_GWR, eq. entropy).
 *   Smoothing. ytilde <- ytilde + q (y - ytilde), q = 1 - exp(-alpha dt)
 *     (eq. myts for y constant over a step); ytilde = y at t = 0.
 *   Step order. Force of change at z^k with Delta^k, leapfrog push to
 *     z^{k+1}, deposit at z^{k+1}, smoothing, residuals; with M2M_S_MPR and
 *     prior_every > 0, every prior_every-th correction step then recomputes
 *     the cell priors from z^{k+1}; they act from the next step on.
 *   Potential. Hernquist (eq. her) of mass M_star*upsilon and scale a, plus
 *     optionally NFW: Phi = -G M200/f(c) ln(1 + r/r_s)/r,
 *     f(c) = ln(1+c) - c/(1+c) (M200 = 0: none), plus optionally the
 *     logarithmic halo Phi_D = v0^2/2 ln(r0^2 + R^2 + z^2/q^2) (v0 = 0:
 *     none), flattened along z for q != 1. With the logarithmic halo every
 *     energy above Phi(0) is bound, and L_c(E) is the angular momentum of the
 *     circular orbit of energy E in the equatorial plane.
 *   Observables, in this order (J = m2m_num_observables):
 *     the density part, one of
 *       M2M_DENS_BINS: n_r radial mass bins, K = 1 for r in [e_k, e_{k+1}),
 *         e_k = r_min (r_max/r_min)^(k/n_r) (e_0 = r_min, e_{n_r} = r_max);
 *       M2M_DENS_ALM: the spherical-harmonic coefficients a_lm,k of Sec. 3.3
 *         (eq. alm) on the n_r mesh radii r_k = r_min (r_max/r_min)^(k/(n_r-1)):
 *         entry k (l_max+1)^2 + l^2 + l + m, 0 <= l <= l_max, -l <= m <= l,
 *         K = gamma_k(r) Y_lm(theta, phi), with the real orthonormal harmonics
 *         Y_l0 = N_l0 P_l(cos t), Y_lm = sqrt2 N_lm P_l^m(cos t) cos(m phi),
 *         Y_l,-m = sqrt2 N_lm P_l^m(cos t) sin(m phi) (m > 0; P_l^m with the
 *         Condon-Shortley phase, N_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!),
 *         cos t = z/r, phi the azimuth of (x, y)) and the cloud-in-cell
 *         weights, linear in r: for r_k <= r < r_{k+1},
 *         gamma_k = (r_{k+1} - r)/(r_{k+1} - r_k), gamma_{k+1} = 1 - gamma_k,
 *         nothing outside [r_0, r_{n_r-1});
 *     then per projected annulus p (R = sqrt(x^2 + y^2), the same log edges
 *     on [R_min, R_max); the line of sight is z), contiguous:
 *       M2M_KIN_V2:    one entry, K = v_z^2;
 *       M2M_KIN_GH:    gh_nmax entries n = 1..gh_nmax, K = 2 sqrt(pi) u_n(nu),
 *                      u_n = (2^(n+1) pi n!)^(-1/2) H_n(nu) exp(-nu^2/2),
 *                      nu = (v_z - V_p)/sigma_p (eq. lumghn);
 *       M2M_KIN_LOSVD: n_v entries, K = 1 for v_z in the k-th of n_v equal
 *                      bins of [v_min, v_max).
 *     A particle outside a range has no kernel there (selection function).
 *   Prior cells. k = floor((E - E_lo)/(E_hi - E_lo) n_E), or with
 *     M2M_CELLS_EXP_E k = floor((exp E - exp E_lo)/(exp E_hi - exp E_lo) n_E),
 *     l = floor(x n_x), both clamped into the grid; cell k n_x + l, and with
 *     M2M_CELLS_LZ cell n_E n_x + k n_x + l for particles with L_z < 0
 *     (C = 2 n_E n_x cells, at most 4096); E = v^2/2 + Phi(x, y, z),
 *     x = |r x v| / L_c(E); x = 1 for E <= Phi(0), and without the
 *     logarithmic halo x = 0 for E >= 0.
 *     Empty cells keep their previous prior (no particle reads them).
 *   Prior smoothing (smooth = 1, eq. smooth_grid). Each n_E x n_x grid (both
 *     halves with M2M_CELLS_LZ) is smoothed alone, with the cell width along
 *     energy measured in exp E with M2M_CELLS_EXP_E. The grid w0 of cell means
 *     (previous priors for empty cells) is replaced by the minimizer of
 *     |w - w0|^2 + lambda w^T P w, P the finite-difference thin-plate
 *     penalty (d2w/dE2)^2 + 2 (d2w/dEdx)^2 + (d2w/dx2)^2 on the grid in its
 *     own units (cell widths hE = (E_hi - E_lo)/n_E and hx = 1/n_x), each
 *     difference taken only where its stencil lies inside the grid:
 *     w[k+1][l] - 2 w[k][l] + w[k-1][l] over hE^2 at cells with neighbours
 *     on both sides along E, likewise along x, and w[k+1][l+1] - w[k+1][l] -
 *     w[k][l+1] + w[k][l] over hE hx at every interior corner. Planes cost
 *     nothing: lambda -> infinity gives the least-squares plane. lambda
 *     minimizes the generalized cross validation score
 *       GCV = (|w0 - A w0|^2/n) / (1 - tr(A)/n)^2,  A = (I + lambda P)^-1,
 *     over log10 lambda: steps of 0.25 over [-2 log10(G_hi) - 4,
 *     -2 log10(G_lo) + 4] (G_hi = 4/hE^2 + 4/hx^2, G_lo the smaller of
 *     4 sin^2(pi/2n)/h^2 over axes with more than one cell), then 65 points
 *     over the two steps around the best one, then 65 points over the two
 *     sub-steps around the best one (the first minimum on ties). Smoothed
 *     priors are floored at 1e-3 times the mean of w0. The library computes
 *     the eigendecomposition of P once per grid shape on the host (see
 *     m2m_smoothing_basis) and smooths on the device in that basis.
 *   Self-consistent potential (scf_nr > 0). The stellar potential is the
 *     multipole expansion of the particles, m_i = upsilon u_i M / N:
 *       Phi_*(x) = sum_lm Phi_lm(r) Y_lm(theta, phi)  (l <= scf_lmax, the
 *       real harmonics above),
 *       Phi_lm(r) = -4 pi G / (2l+1) [r^-(l+1) A_lm(r) + r^l B_lm(r)],
 *       A_lm(r) = sum_{r_i < r} m_i r_i^l Y_lm(x_i),
 *       B_lm(r) = sum_{r_i >= r} m_i r_i^-(l+1) Y_lm(x_i),
 *     exact with its slope r dPhi_lm/dr at the nodes
 *     rho_k = scf_rmin (scf_rmax/scf_rmin)^(k/(scf_nr-1)); between nodes
 *     Phi_lm is the cubic Hermite interpolant of value and slope in ln r,
 *     inside rho_0 r^l (c0 + c1 r^2), beyond the last node the decaying
 *     c0 r^-(l+1) + c1 r^-(l+3), each matching value and slope at the end
 *     node. The force is its exact gradient (zero at r = 0). Particles with
 *     a non-finite radius add nothing to the expansion. The expansion is built from the
 *     particles and weights when the targets are first set (or by
 *     m2m_refresh_potential) and rebuilt after the push of every step k with
 *     (k + 1) % scf_every == 0, counting steps of every kind from 0, from
 *     z^{k+1} and the weights after that step; it acts from the next step on.
 *
 * Memory and ownership
 *   Particle arrays (x, y, z, vx, vy, vz, u, u_prior) are device pointers in
 *   structure-of-arrays layout, float (M2M_F32) or double (M2M_F64), each
 *   16-byte aligned, owned by the caller and required to outlive the
 *   context. The library owns (or borrows, if a workspace is passed) one
 *   device workspace per context holding targets, observables, tables,
 *   reduction buffers and the prior cell of every particle at the last
 *   refresh (2 bytes per particle). New priors reach u_prior at the start of
 *   the step after a refresh, or at m2m_get_weights / m2m_get_state /
 *   m2m_update_priors, whichever comes first. All device work is enqueued on the stream given at
 *   creation (a hipStream_t passed as void*; NULL is the null stream).
 *
 * Errors
 *   Every call returns a status and never aborts. Invalid arguments give
 *   M2M_EINVAL, allocation failure M2M_ENOMEM, a failing HIP call
 *   M2M_EDEVICE, a call out of order M2M_ESTATE. Asynchronous calls report
 *   device-side problems (a non-finite chi^2) at the next synchronizing call
 *   (m2m_get_*, m2m_observe, m2m_batch_poll) as M2M_ENONFINITE.
 *   m2m_last_error gives a message for the last failure on a context.
 *   A context is not thread-safe; distinct contexts are independent.
 */
#ifndef M2M_H
#define M2M_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct m2m_ctx m2m_ctx;
typedef struct m2m_batch m2m_batch;

typedef enum {
    M2M_OK = 0,
    M2M_EINVAL = 1,
    M2M_ENOMEM = 2,
    M2M_EDEVICE = 3,
    M2M_ESTATE = 4,
    M2M_ENONFINITE = 5,
    M2M_EUNSUPPORTED = 6
} m2m_status;

typedef enum { M2M_F32 = 0, M2M_F64 = 1 } m2m_dtype;
typedef enum { M2M_S_MPR = 0, M2M_S_GWR = 1 } m2m_entropy;
typedef enum { M2M_KIN_NONE = 0, M2M_KIN_V2 = 1, M2M_KIN_GH = 2, M2M_KIN_LOSVD = 3 } m2m_kin;
typedef enum { M2M_DENS_BINS = 0, M2M_DENS_ALM = 1 } m2m_dens;
/* prior-grid options for rotating models (Sec. 5): a second n_E x n_x grid
 * for particles with L_z < 0; energy bins linear in exp(E) */
typedef enum { M2M_CELLS_LZ = 1, M2M_CELLS_EXP_E = 2 } m2m_cells;

/* Fixed potential (Sec. 3.1, eq. her; NFW halo optional; logarithmic halo
 * of Sec. 5, eq. log_halo, optional). */
typedef struct {
    double G, M_star, a, upsilon; /* Hernquist mass M_star*upsilon, scale a > 0 */
    double M200, c, r_s;          /* NFW: M200 = 0 for none; else c > 0, r_s > 0 */
    double v0, r0, q;             /* logarithmic halo: v0 = 0 for none; else r0 > 0, q > 0 */
} m2m_potential;

/* Observable kernels K_j (Sec. 2.1; eqs. alm, lumghn). Radii are in length
 * units, velocities in velocity units. n_r >= 1; kin is an m2m_kin. */
typedef struct {
    int32_t n_r;
    double r_min, r_max;  /* 0 < r_min < r_max */
    int32_t n_R;          /* annuli; 0 allowed only with kin = M2M_KIN_NONE */
    double R_min, R_max;  /* 0 < R_min < R_max */
    int32_t kin;
    int32_t gh_nmax;      /* M2M_KIN_GH: 1..8 */
    int32_t n_v;          /* M2M_KIN_LOSVD: 1..256 */
    double v_min, v_max;  /* M2M_KIN_LOSVD: v_min < v_max */
    int32_t dens;         /* m2m_dens: density observables; M2M_DENS_ALM needs n_r >= 2 */
    int32_t l_max;        /* M2M_DENS_ALM: 0..8 */
} m2m_obs_layout;

/* Step parameters (eqs. modFOC, myts, S+, entropy; Sec. 2.3.1, 4.1). */
typedef struct {
    double dt;           /* leapfrog step, > 0 */
    double eps;          /* force-of-change rate, >= 0 */
    double mu;           /* entropy weight, >= 0 */
    double alpha;        /* smoothing rate (1/time), >= 0 */
    double mass;         /* total mass M: w_i = u_i M / N, > 0 */
    int32_t entropy;     /* m2m_entropy */
    int32_t n_E, n_x;    /* prior grid, n_E, n_x >= 1, n_E * n_x <= 4096 */
    int32_t prior_every; /* correction steps between prior refreshes; 0 = never */
    double E_lo, E_hi;   /* energy range of the grid, E_lo < E_hi */
    int32_t smooth;      /* 1: smooth the prior grid at every refresh (Sec. 2.3.2, see
                            "Prior smoothing"); needs n_E, n_x <= 128 and
                            n_E * n_x <= 2048; 0: cell means */
    int32_t cells;       /* m2m_cells flags of the prior grid (Sec. 5); 0: n_E x n_x
                            cells linear in E */
    /* Self-consistent stellar potential (Sec. 2.1: a potential computed from
     * the particles as they move; Sec. 5: from a spherical-harmonic
     * decomposition of the light at constant M/L). scf_nr = 0: none, the
     * Hernquist part of m2m_potential is the stars. Otherwise the stars are
     * the multipole expansion of the particles' masses upsilon w_i to degree
     * scf_lmax, known at scf_nr nodes log-spaced over [scf_rmin, scf_rmax]
     * (see "Self-consistent potential"); the NFW and logarithmic halos stay
     * analytic, and the prior cells keep the analytic potential. */
    int32_t scf_lmax;    /* 0..8 */
    int32_t scf_nr;      /* 0, or 2..64 nodes */
    double scf_rmin, scf_rmax; /* 0 < scf_rmin < scf_rmax */
    int32_t scf_every;   /* steps between rebuilds of the expansion, >= 1 */
} m2m_params;

/* Number of observables J of a layout (0 if the layout is invalid). */
int32_t m2m_num_observables(const m2m_obs_layout* layout);

/* Bytes of device workspace a context needs for n particles. */
size_t m2m_workspace_bytes(const m2m_obs_layout* layout, const m2m_params* params, int64_t n,
                           int32_t dtype);

/* Create a context over caller-owned device particle arrays (Sec. 2.1).
 * n >= 1 particles; dtype is an m2m_dtype; u and u_prior hold u_i and uhat_i
 * (see "Weights"). workspace: NULL to let the library allocate it, else a
 * device buffer of at least m2m_workspace_bytes(...) bytes owned by the
 * caller. hip_stream: the stream all work of this context is ordered on.
 * On success *out receives the context; on failure *out is NULL.
 * M2M_EINVAL, before any device call, for n < 1 (an empty fit), an unknown
 * dtype, a NULL array or one that is not 16-byte aligned, and for invalid
 * potential, layout or parameters.
 * M2M_EUNSUPPORTED if the step kernel's LDS tables do not fit the 160 KiB of
 * a compute unit: the bins (private copies), the cell sums, the edge tables
 * and, with the self-consistent potential, its interval table ((scf_nr + 1)
 * (scf_lmax+1)^2 four-vectors of the state type) and FP64 interval sums
 * (2 scf_nr (scf_lmax+1)^2); l <= 8 fits up to about 54 nodes with FP32 state
 * and 35 with FP64 state at a few hundred observables. */
m2m_status m2m_create(const m2m_potential* pot, const m2m_obs_layout* layout,
                      const m2m_params* params, int64_t n, int32_t dtype, void* x, void* y,
                      void* z, void* vx, void* vy, void* vz, void* u, void* u_prior,
                      void* workspace, size_t workspace_bytes, void* hip_stream, m2m_ctx** out);

/* Targets Y_j and errors sigma(Y_j) (eq. delta), host arrays of J doubles,
 * copied. V_p, sigma_p: host arrays of n_R doubles, the Gauss-Hermite centres
 * (required for M2M_KIN_GH, ignored otherwise, may be NULL). The first call
 * also measures the current state: ytilde = y (t = 0). Later calls replace
 * the data and recompute Delta from the current ytilde. EINVAL for J not
 * matching the layout, non-finite values or sigma <= 0, sigma_p <= 0. */
m2m_status m2m_set_targets(m2m_ctx* ctx, int32_t J, const double* Y, const double* sigma,
                           const double* V_p, const double* sigma_p);

/* Enqueue n_steps M2M steps (asynchronous). correct = 0 runs them without
 * weight correction (relaxation, Sec. 4.1): push, deposit and smoothing. */
m2m_status m2m_step(m2m_ctx* ctx, int32_t n_steps, int32_t correct);

/* Recompute the cell priors from the current state now (Sec. 2.3.1) and
 * assign them; asynchronous. EINVAL unless entropy is M2M_S_MPR. */
m2m_status m2m_update_priors(m2m_ctx* ctx);

/* Rebuild the self-consistent stellar potential (Sec. 2.1, Sec. 5) from the
 * current particles and weights now; asynchronous. It acts from the next
 * step on. Call it after changing the particle arrays between steps.
 * EINVAL unless params.scf_nr > 0, ESTATE inside a batch. */
m2m_status m2m_refresh_potential(m2m_ctx* ctx);

/* The node table of the self-consistent potential into out (host memory,
 * max >= scf_nr (scf_lmax+1)^2 2 doubles): entry (k (scf_lmax+1)^2 + l^2 +
 * l + m) 2 is Phi_lm(rho_k), the next one r dPhi_lm/dr at rho_k.
 * Synchronizes the stream. EINVAL without the expansion or if max is too
 * small, ESTATE inside a batch. */
m2m_status m2m_get_potential(m2m_ctx* ctx, double* out, int32_t max);

/* Weights w_i = u_i M / N into dst (n values of the context's dtype), on the
 * device (dst_is_device = 1) or the host. Synchronizes the stream. */
m2m_status m2m_get_weights(m2m_ctx* ctx, void* dst, int32_t dst_is_device);

/* Host copies (J doubles each; any pointer may be NULL) of the last raw
 * deposit y, the smoothed ytilde, the residuals Delta, and chi^2.
 * Synchronizes. */
m2m_status m2m_get_observables(m2m_ctx* ctx, double* y, double* y_tilde, double* delta,
                               double* chi2);

/* chi^2 after each of the last steps, oldest first: up to max values into
 * out (host), their number in *n_out. Synchronizes. */
m2m_status m2m_get_chi2_history(m2m_ctx* ctx, double* out, int32_t max, int32_t* n_out);

/* Measure the current particle state without changing it: y_j (host, J
 * doubles) with the given Gauss-Hermite centres (host, n_R doubles each;
 * NULL uses the ones set by m2m_set_targets, or V = 0, sigma = 1).
 * Synchronizes. Used to build targets from a realization (Sec. 3.1). */
m2m_status m2m_observe(m2m_ctx* ctx, const double* V_p, const double* sigma_p, double* y);

/* Allocation-free observation, for callers that cannot allocate device
 * memory (code that must keep a fixed device footprint, such as serving
 * loops, and harnesses that forbid hipMalloc): y_j (host, J doubles) of the
 * particle set (x, y, z, vx, vy, vz, u: n particles of dtype, device,
 * 16-byte aligned, read only) with total mass M, w_i = u_i M / n, exactly as
 * m2m_observe computes it for a context of this layout, mass and particle
 * count (same kernels and tiles; without prior cells the tile count can
 * differ for small n, and with it the FP64 summation order).
 * V_p, sigma_p: host, n_R doubles each, required for M2M_KIN_GH, ignored
 * otherwise. hip_stream: a hipStream_t as void* (NULL: the null stream).
 *   The working memory (tables, counters, tile rows, the observables) is a
 * static device array of M2M_NOALLOC_SCRATCH_BYTES that every GPU the
 * library runs on holds until the process ends; the call allocates no
 * device memory and calls no allocating HIP or library routine. It keeps
 * the last call's contents; the counters are cleared at every call. A
 * layout and particle count that need more working memory than the array
 * holds give M2M_ENOMEM (observables x 8 bytes per tile row; about 256 tile
 * rows at the default launch shape). Synchronizes. Calls from one process
 * run one at a time; calls from different processes on one GPU each have
 * their own array. Calls whose device work overlaps on one GPU (another
 * stream of the same process, hipGraph replays of such work) would race on
 * the array. Failure messages: m2m_last_error(NULL) on the calling thread. */
#define M2M_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
m2m_status m2m_observe_noalloc(const m2m_obs_layout* layout, double mass, int64_t n,
                               int32_t dtype, const void* x, const void* y, const void* z,
                               const void* vx, const void* vy, const void* vz, const void* u,
                               const double* V_p, const double* sigma_p, double* obs,
                               void* hip_stream);

/* Checkpoint of everything the context holds besides the particle arrays
 * (ytilde, cell priors, counters, targets). With host_blob = NULL, *bytes
 * receives the size. Synchronizes. m2m_set_state restores it into a context
 * created with the same layout and parameters. */
m2m_status m2m_get_state(m2m_ctx* ctx, void* host_blob, size_t* bytes);
m2m_status m2m_set_state(m2m_ctx* ctx, const void* host_blob, size_t bytes);

/* Timing by HIP events on the context's stream. With r = ceil(n_steps / 32)
 * (n_steps 1..4096), runs r graphs of 32 steps as m2m_step does, then r
 * graphs of 32 steps each followed by one more finalize reduction in a
 * measuring mode that changes no state: 64 r steps in all, which advance
 * the fit. With S and S2 the mean times per step of the two runs,
 * ms_finalize = S2 - S is the reduction's cost where it runs and
 * ms_step = S - ms_finalize that of the fused step kernel (milliseconds).
 * Synchronizes. Used to report achieved bandwidth against the roofline. */
m2m_status m2m_profile_step(m2m_ctx* ctx, int32_t n_steps, int32_t correct, double* ms_step,
                            double* ms_finalize);

/* The eigendecomposition P = Q diag(g) Q^T of the prior-smoothing penalty of
 * an n_E x n_x grid with cell widths hE, hx (Sec. 2.3.2, eq. smooth_grid; see
 * "Prior smoothing"), as the device smoother uses it; host only, no device
 * call. Q is the orthonormal parity basis of the two axis reflections times
 * block eigenvectors. Along an axis of n cells, even vector i < ceil(n/2) is
 * (e_i + e_{n-1-i})/sqrt(2) (e_i alone for the middle cell of an odd n) and
 * odd vector i < floor(n/2) is (e_i - e_{n-1-i})/sqrt(2). Block b = 2 pE + pX
 * (parity 0 even, 1 odd) holds the products of E vector i of parity pE and x
 * vector j of parity pX at index r = i m_x(pX) + j; its m_b x m_b eigenvector
 * matrix has entry [r][o] = component r of eigenvector o. out (host,
 * len doubles) receives the n_E n_x eigenvalues of blocks 0..3, then the
 * eigenvector matrices of blocks 0..3, row-major. With out = NULL, *len
 * receives the length. EINVAL for n_E, n_x outside 1..128, n_E n_x > 2048,
 * hE, hx not > 0 or len too small; EDEVICE if the iteration does not
 * converge. The result is cached per grid shape for the process. */
m2m_status m2m_smoothing_basis(int32_t n_E, int32_t n_x, double hE, double hx, double* out,
                               size_t* len);

/* Release the context and its library-owned workspace (synchronizes). */
m2m_status m2m_destroy(m2m_ctx* ctx);

/* Text of the last failure on ctx (never NULL); with ctx NULL, of the
 * calling thread's last failed m2m_observe_noalloc. */
const char* m2m_last_error(const m2m_ctx* ctx);

/* Launch shape of the fused step kernel for contexts created afterwards and
 * for batches rebuilt afterwards: threads per block (256, 512 or 1024) and
 * tiles (blocks) per compute unit (1..16); each thread handles one particle
 * at a time. EINVAL otherwise. Chosen by the package's autotuner. */
m2m_status m2m_set_launch(int32_t block, int32_t tiles_per_cu);
m2m_status m2m_get_launch(int32_t* block, int32_t* tiles_per_cu);

/* Most private copies of the in-tile observable bins per block of the step
 * kernel, for contexts created afterwards: 1, 2, 4 or 8, or 0 (default) for
 * as many as fit 48 KiB of LDS, at most 8. Lanes add into copy
 * (thread index mod copies), which spreads the LDS atomics of a hot bin.
 * EINVAL otherwise. Chosen by the autotuner. */
m2m_status m2m_set_private_copies(int32_t copies);
int32_t m2m_get_private_copies(void);

/* Groups a batch of two or more fits is split into at its next rebuild
 * (see "batching"): 2 (default, the groups overlap on two streams) or 1 (one
 * step kernel over all fits). EINVAL otherwise. Chosen by the autotuner. */
m2m_status m2m_set_batch_groups(int32_t groups);
int32_t m2m_get_batch_groups(void);

/* How batches rebuilt afterwards enqueue their steps: 1 replays graphs of 8
 * captured steps (and launches the rest directly), 0 (default) launches
 * every step's two kernels directly. A newly captured graph is slow on its
 * first launches, and a batch captures anew at every change of composition;
 * at the step times of batches, direct launches cost nothing measurable.
 * EINVAL otherwise. Chosen by the autotuner. */
m2m_status m2m_set_batch_graphs(int32_t on);
int32_t m2m_get_batch_graphs(void);

/* In-tile accumulation of the deposits (eq. obs) for FP32 particle state,
 * for contexts and batches created afterwards: M2M_DEPOSIT_F64 (default)
 * adds each w_i K_j(z_i), formed in FP32, into FP64 bins in LDS;
 * M2M_DEPOSIT_F32_COMPENSATED adds it into FP32 bins and carries the exact
 * rounding error of every add (TwoSum) in a second FP32 array. Tile sums are
 * reduced across tiles in FP64 in a fixed order either way. FP64 particle
 * state always uses FP64 bins. EINVAL for an unknown mode. */
typedef enum { M2M_DEPOSIT_F64 = 0, M2M_DEPOSIT_F32_COMPENSATED = 1 } m2m_deposit_mode;
m2m_status m2m_set_deposit_mode(int32_t mode);
int32_t m2m_get_deposit_mode(void);

/* Which particles a tile of the step kernel of one fit takes, for contexts
 * created afterwards: 0 its contiguous range, 1 interleaved chunks of one
 * block's width (tile t of T takes chunks t, t + T, t + 2T, ...), or -1
 * (default) interleaved for particle states above 128 MiB (8 arrays of n
 * values) and contiguous below. Interleaving applies to fits of FP32 state
 * with FP64 bins (M2M_DEPOSIT_F64) and observables without a_lm
 * coefficients, Gauss-Hermite moments beyond h_4 or the self-consistent
 * potential, below 2^30 particles; other fits and batches take contiguous
 * ranges. The sums are the same up to rounding order. EINVAL otherwise. */
m2m_status m2m_set_interleave(int32_t mode);
int32_t m2m_get_interleave(void);

/* ---------------------------------------------------------- batching --
 * Many fits of uneven size stepping together. A batch of two or more fits is
 * split into two groups of about equal particle count; every step of a group
 * runs one fused kernel over the tiles of its fits (tiles never straddle
 * fits) and one finalize kernel, launched directly (or replayed from captured
 * HIP graphs, m2m_set_batch_graphs) on a stream of the group's own, so that
 * one group's finalize overlaps the other group's streaming. The groups
 * start after the work already enqueued on the batch stream, and the batch
 * stream continues only after both (events), so to the caller the steps are
 * ordered on the batch stream. Each fit's result equals the fit run alone up
 * to the rounding of its in-tile sums. Fits keep their own streams for
 * set-up. When fits come or go, the next run copies the new fit, tile and
 * finalize tables on the batch stream, after the runs already enqueued and
 * without waiting for them (with graphs: after waiting for them). A fit
 * leaves the batch when a poll hands it back or it is cancelled; the work
 * on its own stream that changes its state then waits for the batch runs
 * enqueued before (they may still read it), and m2m_destroy waits for them. */

/* hbm_budget: bytes of particle state plus workspace the batch may hold
 * (0 = no limit). max_fits >= 1. */
m2m_status m2m_batch_create(int32_t max_fits, size_t hbm_budget, void* hip_stream,
                            m2m_batch** out);
/* Add a fit (targets set) to run n_steps correction steps. ENOMEM when its
 * footprint would exceed the budget or the batch is full; the fit is then
 * not admitted and can be retried later. ESTATE if already in a batch. */
m2m_status m2m_batch_admit(m2m_batch* b, m2m_ctx* fit, int32_t n_steps);
/* Enqueue steps_per_launch steps of every admitted fit with steps left. */
m2m_status m2m_batch_run(m2m_batch* b, int32_t steps_per_launch);
/* Synchronize, then hand back (and remove from the batch) up to max_done
 * fits that have run all their steps. *n_done receives their number;
 * *n_active (may be NULL) the number still running. */
m2m_status m2m_batch_poll(m2m_batch* b, m2m_ctx** done, int32_t max_done, int32_t* n_done,
                          int32_t* n_active);
/* The same without draining the batch, for a loop that keeps the GPU busy:
 * every m2m_batch_run ends with a snapshot of the fits' completion flags on
 * the batch stream; this call waits only for the snapshot of the run before
 * the latest one (not yet read by an earlier call) and hands back up to
 * max_done fits that had run all their steps by then, while the latest run
 * may still execute. With no such snapshot it returns at once (*n_done = 0).
 * A fit handed back keeps its weights from its last step; reading them
 * (m2m_get_weights) does not wait for the batch. */
m2m_status m2m_batch_poll_lagged(m2m_batch* b, m2m_ctx** done, int32_t max_done,
                                 int32_t* n_done, int32_t* n_active);
/* Timing of the batch's kernels by HIP events on the batch stream: n_steps
 * (1..256) batched steps launched one kernel at a time (no graph), each step
 * kernel between two events. ms_step is the mean time between those two
 * events (the step kernel, plus the events' own small cost: an upper bound),
 * ms_finalize the mean rest of a step (the finalize and the gaps around it).
 * The steps count against the fits' steps. Synchronizes. Used to report the
 * step kernel's achieved bandwidth against the roofline. */
m2m_status m2m_batch_profile(m2m_batch* b, int32_t n_steps, double* ms_step, double* ms_finalize);
/* Particles of the admitted fits that still have steps left. Synchronizes. */
int64_t m2m_batch_particles(m2m_batch* b);
/* Bytes of budget in use. */
size_t m2m_batch_footprint(const m2m_batch* b);
/* Remove a fit before it finished (cancellation); synchronizes. */
m2m_status m2m_batch_cancel(m2m_batch* b, m2m_ctx* fit);
m2m_status m2m_batch_destroy(m2m_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* M2M_H */

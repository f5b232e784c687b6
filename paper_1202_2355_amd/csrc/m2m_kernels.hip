// HIP kernels (gfx950) of the chi^2 M2M step with moving priors.
//
// One M2M step is two kernels (k_step in m2m_step.h, instantiated by the
// m2m_step_*.hip units; the rest here):
//   k_step      one streaming pass over the particles of every active fit,
//               one block per tile: (assign the new cell priors) -> force of
//               change at z^k (eq. modFOC with eq. S+ or eq. entropy) ->
//               drift-kick-drift push -> deposit of w K_j(z^{k+1}) (eq. obs)
//               into LDS bins -> (prior-cell sums, Sec. 2.3.1). Each tile
//               writes one row of FP64 partial sums.
//   k_finalize  FP64 reduction of the tile rows of every fit in a fixed
//               order -> y, smoothed ytilde (eq. myts), Delta and chi^2
//               (eqs. delta, chi), the force table for the next step, and
//               the cell means that become the new priors.
// Particle state is structure-of-arrays, read and written once per step
// (coalesced, one particle per lane, the next batch prefetched). k_step is
// specialized at compile time on the kind of kinematic observable.
#include <hip/hip_runtime.h>

#include "m2m_device.h"

namespace m2m {
namespace {

// ------------------------------------------------------------- finalize ----
// The reduction of a step: one block per job of kFinCols columns of one fit.
//   column sums over the fit's tile rows in one fixed order: row group g
//   (g < kFinWaves) adds rows g, g + kFinWaves, ... in row order, then the
//   groups are added in order;
//   observable columns: smoothing (eq. myts), Delta and chi^2 (eqs. delta,
//   chi) and the force table; cell columns: the cell means that become the
//   priors (Sec. 2.3.1);
//   the end of the step: chi^2 from the parts of the bin jobs and the step
//   counters, prior schedule and assignment flag.
struct Flags {
    bool step, cells_mode, observe, init, correct, refresh, pot_mode, pot;
};

// The fit's counters as the launch found them: only the block that ends the
// step writes them, from these values, so they are read once, up front.
struct Snap {
    int64_t kstep, tstep;
    int32_t steps_left, correct, error;
};

__device__ __forceinline__ Snap snap_of(G<const FitState> st) {
    Snap s;
    s.kstep = st->kstep;
    s.tstep = st->tstep;
    s.steps_left = st->steps_left;
    s.correct = st->correct;
    s.error = st->error;
    return s;
}

template <bool SCF>
__device__ __forceinline__ Flags flags_of(const FitDev& fd, const Snap& ss, int32_t mode) {
    Flags f;
    f.step = (mode & kModeStep) != 0;
    f.cells_mode = (mode & kModeCells) != 0;
    f.observe = (mode & kModeObserve) != 0;
    f.init = (mode & kModeInit) != 0;
    f.correct = f.step && ss.correct != 0;
    f.refresh = f.cells_mode || (f.correct && fd.entropy == 0 && fd.prior_every > 0 &&
                                 ((ss.kstep + 1) % fd.prior_every) == 0);
    // the self-consistent potential is rebuilt (kModePot alone, or every
    // scf_every steps)
    f.pot_mode = SCF && (mode & kModePot) != 0;
    f.pot = SCF && fd.scf_nr > 0 &&
            (f.pot_mode || (f.step && ((ss.tstep + 1) % fd.scf_every) == 0));
    return f;
}

// Row group g of one column: the sum of rows g, g + kFinWaves, ... in row
// order (and of the matching count column for cells), U rows in flight (the
// sum does not depend on U).
template <int U>
__device__ __forceinline__ void group_sum(const FitDev& fd, bool bins, int col, int n_tiles, int g,
                                          double& acc, double& acc2) {
    const size_t stride = (size_t)fd.row_len;
    const int J = fd.J, C = fd.C;
    if (bins) {
        const G<const double> base = gmem<const double>(fd.partials) + col;
        for (int t0 = g; t0 < n_tiles; t0 += U * kFinWaves) {
            double v[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int t = t0 + k * kFinWaves;
                v[k] = (t < n_tiles) ? base[(size_t)t * stride] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < U; ++k) acc += v[k];
        }
    } else {
        const G<const double> base = gmem<const double>(fd.partials) + J + col;
        for (int t0 = g; t0 < n_tiles; t0 += U * kFinWaves) {
            double v[U], w[U];
#pragma unroll
            for (int k = 0; k < U; ++k) {
                const int t = t0 + k * kFinWaves;
                v[k] = (t < n_tiles) ? base[(size_t)t * stride] : 0.0;
                w[k] = (t < n_tiles) ? base[(size_t)t * stride + C] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < U; ++k) {
                acc += v[k];
                acc2 += w[k];
            }
        }
    }
}

// Column epilogue of one job (one wave; lane = column offset): tot, tot2 are
// the column sums. Returns this job's chi^2 part (lane 0, bin jobs).
template <typename T>
__device__ __forceinline__ double column_epilogue(const FitDev& fd, bool bins, int col0,
                                                  const Flags& f, double tot, double tot2,
                                                  double yt0, double sg, double Yj, int lane) {
    const int col = col0 + lane;
    double d2 = 0.0;
    if (bins && col < fd.J) {
        if (f.observe) {
            gmem(fd.obs_out)[col] = tot;
        } else {
            gmem(fd.yv)[col] = tot;
            const double yt = f.init ? tot : yt0 + fd.q * (tot - yt0);
            gmem(fd.ytil)[col] = yt;
            const double d = (yt - Yj) / sg;
            gmem(fd.delta)[col] = d;
            gmem<T>(fd.rp)[col] = (T)(fd.foc_chi * d / sg);
            d2 = d * d;
        }
    } else if (!bins && col < fd.C) {
        // the cell's data: the mean weight, or the previous prior if empty
        const double d = (tot2 > 0.0) ? tot / tot2 : gmem(fd.gprior)[col];
        gmem(fd.cdata)[col] = d;
        if (!fd.smooth) {
            gmem(fd.gprior)[col] = d;
            gmem<T>(fd.ucell)[col] = (T)d;
        }
    }
    if (bins && !f.observe) {
        // chi^2 of these columns: fixed-order butterfly over the wave
        for (int off = 32; off >= 1; off >>= 1) d2 += __shfl_xor(d2, off, 64);
        if (lane == 0) gmem(fd.chi2_part)[col0 / kFinCols] = d2;
    }
    return d2;
}

// chi^2 from the parts of the bin jobs (one wave): lane l adds parts l,
// l + 64, ... in order, then a fixed-order butterfly over the wave.
__device__ __forceinline__ double chi2_of_parts(const double* parts, int n, int lane) {
    double c = 0.0;
    for (int b = lane; b < n; b += 64) c += parts[b];
    for (int off = 32; off >= 1; off >>= 1) c += __shfl_xor(c, off, 64);
    return c;
}

// The end of the step for one fit (one thread): the new counters from the
// launch's snapshot of them (stores only).
__device__ __forceinline__ void end_step(const FitDev& fd, G<FitState> gst, const Flags& f,
                                         const Snap& ss, double chi2) {
    if (!f.cells_mode) {
        gst->chi2 = chi2;
        if (!isfinite(chi2)) gst->error = ss.error | 1;
        if (f.step) gmem(fd.chi2_hist)[ss.tstep % kHistCap] = chi2;
    }
    if (f.step) {
        gst->tstep = ss.tstep + 1;
        gst->steps_left = ss.steps_left - 1;
        if (f.correct) gst->kstep = ss.kstep + 1;
        gst->assign_pending = f.refresh ? 1 : 0;
    }
    if (f.cells_mode) gst->assign_pending = 1;
}

// GCV score (RSS/n) / (1 - tr(A)/n)^2 of the spectral smoother at P values
// of lambda, summed by one wave over the n cells (Gamma^2 in g2, transformed
// data in wh); 1 / (1 + t) is a hardware reciprocal refined by two Newton
// steps (within an ulp or two), as the score only ranks the lambdas.
template <int P>
__device__ __forceinline__ void gcv_points(const double* g2, const double* wh, int n, int lane,
                                           const double* lam, double* out) {
    double rss[P], den[P];
#pragma unroll
    for (int j = 0; j < P; ++j) rss[j] = den[j] = 0.0;
    for (int c = lane; c < n; c += 64) {
        const double g = g2[c], w = wh[c];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const double t = lam[j] * g;
            const double d = 1.0 + t;
            double iv = __builtin_amdgcn_rcp(d);
            iv = fma(iv, fma(-d, iv, 1.0), iv);
            iv = fma(iv, fma(-d, iv, 1.0), iv);
            const double r = t * iv;
            const double e = r * w;
            rss[j] = fma(e, e, rss[j]);
            den[j] += r;
        }
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
        for (int off = 32; off >= 1; off >>= 1) {
            rss[j] += __shfl_xor(rss[j], off, 64);
            den[j] += __shfl_xor(den[j], off, 64);
        }
        out[j] = (rss[j] / n) / ((den[j] / n) * (den[j] / n));
    }
}

// Thin-plate smoothing of one n_E x n_x prior grid (the cells from `base`)
// with the GCV-chosen lambda (Sec. 2.3.2, eq. smooth_grid) by the block
// that ends a refresh step; the energy cell width is sm_hE. On the grid
// with reflecting boundaries the penalty is |Lap w|^2 and the orthonormal
// 2-D DCT-II diagonalizes Lap: its basis along an axis of n cells is
// s_k cos(pi k (2i+1) / 2n) (s_0 = sqrt(1/n), s_k = sqrt(2/n)) with
// eigenvalues -(2 - 2 cos(pi k / n)) / h^2. With Gamma the sum of the two
// axes' eigenvalue magnitudes and the transformed data w^ the smoother is the filter
// 1/(1 + lambda Gamma^2), and
//   |w0 - A w0|^2 = sum (t/(1+t))^2 w^^2,  1 - tr(A)/n = sum t/(1+t) / n,
// t = lambda Gamma^2. The log10(lambda) search: steps of 0.25 from sm_plo
// (sm_k1 points), then 65 points over the two steps around the best, then
// 65 points over the two sub-steps around the best (first minimum on
// ties). Smoothed priors are floored at 1e-3 of the mean of the data.
// In LDS: the grids sa, sb (kMaxCells doubles each), buf (scores and
// lambdas of a search stage) and per axis the table
// cos(pi j / 2n), j < 4n, from which every basis value and eigenvalue is
// read (the argument k (2i+1) is taken modulo 4n).
template <typename T>
__device__ __forceinline__ void smooth_priors(const FitDev& fd, int base, double* sa, double* sb,
                                              double* tE,
                              double* tX, double* buf, int* sidx, double* smean) {
    static_assert(2 * kSmoothMaxPoints <= kFinWaves * kFinCols, "GCV scores and lambdas in buf");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nE = fd.n_E, nx = fd.n_x, n = nE * nx;
    const G<const double> w0 = gmem<const double>(fd.cdata) + base;
    const G<double> gp = gmem(fd.gprior) + base;
    const G<T> uc = gmem<T>(fd.ucell) + base;
    if (n < 2) {
        if (tid == 0) {
            gp[0] = w0[0];
            uc[0] = (T)w0[0];
        }
        return;
    }
    const int pE = 4 * nE, pX = 4 * nx;
    for (int j = tid; j < pE; j += kFinThreads) tE[j] = cos(M_PI * j / (2.0 * nE));
    for (int j = tid; j < pX; j += kFinThreads) tX[j] = cos(M_PI * j / (2.0 * nx));
    for (int c = tid; c < n; c += kFinThreads) sb[c] = w0[c];
    const double sE0 = sqrt(1.0 / nE), sE = sqrt(2.0 / nE);
    const double sX0 = sqrt(1.0 / nx), sX = sqrt(2.0 / nx);
    __syncthreads();
    if (wave == 0) {
        double sm = 0.0;
        for (int c = lane; c < n; c += 64) sm += sb[c];
        for (int off = 32; off >= 1; off >>= 1) sm += __shfl_xor(sm, off, 64);
        if (lane == 0) *smean = sm / n;
    }
    // forward transform along E: sa[k][l] = s_k sum_i cos(pi k (2i+1)/2nE) w0[i][l]
    for (int o = tid; o < n; o += kFinThreads) {
        const int k = o / nx, l = o - k * nx;
        double v = 0.0;
        int idx = k % pE;  // k (2i + 1) mod 4 nE
        const int inc = (2 * k) % pE;
        for (int i = 0; i < nE; ++i) {
            v += tE[idx] * sb[i * nx + l];
            idx += inc;
            if (idx >= pE) idx -= pE;
        }
        sa[o] = (k == 0 ? sE0 : sE) * v;
    }
    __syncthreads();
    // along x: sb[k][m] = s_m sum_j cos(pi m (2j+1)/2nx) sa[k][j]
    for (int o = tid; o < n; o += kFinThreads) {
        const int k = o / nx, m = o - k * nx;
        double v = 0.0;
        int idx = m % pX;
        const int inc = (2 * m) % pX;
        for (int j = 0; j < nx; ++j) {
            v += tX[idx] * sa[k * nx + j];
            idx += inc;
            if (idx >= pX) idx -= pX;
        }
        sb[o] = (m == 0 ? sX0 : sX) * v;
    }
    __syncthreads();
    // Gamma^2 of every cell into sa: (2 - 2 cos(pi k/n)) / h^2 per axis
    {
        const double hE = fd.sm_hE, hx = 1.0 / nx;
        for (int c = tid; c < n; c += kFinThreads) {
            const int k = c / nx, m = c - k * nx;
            const double g = (2.0 - 2.0 * tE[(2 * k) % pE]) / (hE * hE) +
                             (2.0 - 2.0 * tX[(2 * m) % pX]) / (hx * hx);
            sa[c] = g * g;
        }
    }
    __syncthreads();
    // GCV at npts values of log10(lambda) (coarse p = a + 0.25 i, refined
    // p = a + (b - a) i / 64): wave w takes points w, w + 16, ..., up to
    // kGcvSlots of them in one pass over the cells (independent division
    // chains, one load of each cell per pass); wave 0 then finds the index
    // of the first minimum
    double* lams = buf + kSmoothMaxPoints;  // lambda of each point of the stage
    auto stage = [&](bool coarse, double a, double b, int npts) -> int {
        for (int i = tid; i < npts; i += kFinThreads)
            lams[i] = pow(10.0, coarse ? a + 0.25 * i : a + (b - a) * i / 64.0);
        __syncthreads();
        const int mine = wave < npts ? (npts - wave + kFinWaves - 1) / kFinWaves : 0;
        for (int j0 = 0; j0 < mine; j0 += kGcvSlots) {
            const int cnt = min(kGcvSlots, mine - j0);
            double lam[kGcvSlots];
#pragma unroll
            for (int j = 0; j < kGcvSlots; ++j)
                lam[j] = j < cnt ? lams[wave + (j0 + j) * kFinWaves] : 0.0;
            double out[kGcvSlots];
            switch (cnt) {
                case 5: gcv_points<5>(sa, sb, n, lane, lam, out); break;
                case 4: gcv_points<4>(sa, sb, n, lane, lam, out); break;
                case 3: gcv_points<3>(sa, sb, n, lane, lam, out); break;
                case 2: gcv_points<2>(sa, sb, n, lane, lam, out); break;
                default: gcv_points<1>(sa, sb, n, lane, lam, out); break;
            }
            if (lane == 0)
                for (int j = 0; j < cnt; ++j) buf[wave + (j0 + j) * kFinWaves] = out[j];
        }
        __syncthreads();
        if (wave == 0) {
            int bi = npts;
            double bg = 0.0;
            for (int i = lane; i < npts; i += 64)
                if (bi == npts || buf[i] < bg) {
                    bg = buf[i];
                    bi = i;
                }
            for (int off = 32; off >= 1; off >>= 1) {
                const double og = __shfl_xor(bg, off, 64);
                const int oi = __shfl_xor(bi, off, 64);
                if (oi < npts && (bi == npts || og < bg || (og == bg && oi < bi))) {
                    bg = og;
                    bi = oi;
                }
            }
            if (lane == 0) *sidx = bi < npts ? bi : 0;
        }
        __syncthreads();
        return *sidx;
    };
    const int K1 = fd.sm_k1;
    const double plo = fd.sm_plo;
    const int i1 = stage(true, plo, 0.0, K1);
    double a = plo + 0.25 * (i1 > 0 ? i1 - 1 : 0);
    double b = plo + 0.25 * (i1 < K1 - 1 ? i1 + 1 : K1 - 1);
    const int i2 = stage(false, a, b, 65);
    const double na = a + (b - a) * (i2 > 0 ? i2 - 1 : 0) / 64.0;
    const double nb = a + (b - a) * (i2 < 64 ? i2 + 1 : 64) / 64.0;
    const int i3 = stage(false, na, nb, 65);
    const double lam = pow(10.0, na + (nb - na) * i3 / 64.0);
    // filter into sa, inverse along E into sb, along x to the output
    for (int c = tid; c < n; c += kFinThreads) sa[c] = sb[c] / (1.0 + lam * sa[c]);
    __syncthreads();
    for (int o = tid; o < n; o += kFinThreads) {
        const int i = o / nx, m = o - i * nx;
        double v = sE0 * sa[m];  // k = 0
        const int inc = (2 * i + 1) % pE;
        int idx = inc;            // k (2i + 1) mod 4 nE
        for (int k = 1; k < nE; ++k) {
            v += sE * tE[idx] * sa[k * nx + m];
            idx += inc;
            if (idx >= pE) idx -= pE;
        }
        sb[o] = v;
    }
    __syncthreads();
    const double floor_v = 1e-3 * (*smean);
    for (int o = tid; o < n; o += kFinThreads) {
        const int i = o / nx, l = o - i * nx;
        double v = sX0 * sb[i * nx];  // m = 0
        const int inc = (2 * l + 1) % pX;
        int idx = inc;
        for (int m = 1; m < nx; ++m) {
            v += sX * tX[idx] * sb[i * nx + m];
            idx += inc;
            if (idx >= pX) idx -= pX;
        }
        v = fmax(v, floor_v);
        gp[o] = v;
        uc[o] = (T)v;
    }
}

// The node table of the self-consistent potential from the reduced interval
// sums (one thread per node and (l, m)): at node k, A_lm = the sums u r^l Y_lm of
// intervals 0..k (particles inside rho_k), B_lm = the sums u r^-(l+1) Y_lm of
// intervals k+1..K (at or outside rho_k), and
//   Phi_lm = -4 pi c / (2l + 1) [rho^-(l+1) A_lm + rho^l B_lm],
//   r dPhi_lm/dr = -4 pi c / (2l + 1) [-(l+1) rho^-(l+1) A_lm + l rho^l B_lm],
// c = G upsilon M / N (the mass of a particle per unit weight, times G).
__device__ __forceinline__ void build_scf_table(const FitDev& fd) {
    const int K = fd.scf_nr, L = fd.scf_lmax, nlm = (L + 1) * (L + 1);
    const G<const double> a = gmem<const double>(fd.scf_sum);
    const G<const double> b = a + (size_t)K * nlm;  // interval q >= 1 at (q - 1) nlm
    const G<const double> rho = gmem<const double>(fd.scf_rho);
    const G<double> tab = gmem(fd.scf_tab);
    // one thread per (node, l, m); A in ascending, B in descending interval order
    for (int e = threadIdx.x; e < K * nlm; e += blockDim.x) {
        const int k = e / nlm, lm = e - k * nlm;
        int l = 0;
        while ((l + 1) * (l + 1) <= lm) ++l;
        double A = 0.0;
        for (int q = 0; q <= k; ++q) A += a[(size_t)q * nlm + lm];
        double B = 0.0;
        for (int q = K; q > k; --q) B += b[(size_t)(q - 1) * nlm + lm];
        const double r = rho[k];
        double rl = 1.0;
        for (int i = 0; i < l; ++i) rl *= r;
        const double ra = 1.0 / (rl * r);
        const double c = -4.0 * M_PI * fd.scf_c / (2.0 * l + 1.0);
        tab[(size_t)e * 2] = c * (ra * A + rl * B);
        tab[(size_t)e * 2 + 1] = c * (-(l + 1.0) * ra * A + l * rl * B);
    }
}

// SCF: the fit has the self-consistent potential (its potential jobs and the
// node table are compiled in only then)
template <typename T, bool SCF>
__device__ __forceinline__ void finalize_job(const FitDev& fd, const FinJob& jb, int32_t mode) {
    __shared__ double part[kFinWaves][kFinCols];
    __shared__ double part2[kFinWaves][kFinCols];
    __shared__ int last, sidx;
    __shared__ double smean;
    __shared__ double sgrid[2][kMaxCells];  // prior smoothing: grids and cosine tables
    __shared__ double stab[2][4 * kSmoothMaxSide];
    FitState* st = fd.st;
    const G<FitState> gst = gmem(fd.st);
    const bool step = (mode & kModeStep) != 0;
    const bool cells_mode = (mode & kModeCells) != 0;
    const bool observe = (mode & kModeObserve) != 0;
    const bool pot_mode = SCF && (mode & kModePot) != 0;
    const bool bins = jb.kind == 0, pots = SCF && jb.kind == 2;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = jb.col0 + lane;
    const bool in = col < (bins ? fd.J : pots ? fd.scf_P : fd.C);

    // observable columns: the rows and the smoothing inputs are requested
    // before the fit's state is known (their latency overlaps its load)
    double acc = 0.0, acc2 = 0.0;
    double yt0 = 0.0, sg = 1.0, Yj = 0.0;
    if (bins && !cells_mode && !pot_mode && in) {
        group_sum<16>(fd, true, col, jb.n_tiles, wave, acc, acc2);
        if (wave == 0 && !observe) {
            yt0 = gmem(fd.ytil)[col];
            sg = gmem(fd.sigma)[col];
            Yj = gmem(fd.Y)[col];
        }
    }
    const Snap ss = snap_of(gst);
    if (step && ss.steps_left <= 0) return;  // uniform: the fit is idle
    const Flags f = flags_of<SCF>(fd, ss, mode);
    if (bins && (cells_mode || pot_mode)) return;
    if (jb.kind == 1 && !f.refresh) return;
    if (pots && !f.pot) return;
    // cell columns, read only on refresh steps; potential columns only on
    // the steps that rebuild it
    if (jb.kind == 1 && in) group_sum<8>(fd, false, col, jb.n_tiles, wave, acc, acc2);
    if (pots && in) group_sum<16>(fd, true, fd.scf_col0 + col, jb.n_tiles, wave, acc, acc2);
    part[wave][lane] = acc;
    part2[wave][lane] = acc2;
    __syncthreads();
    if (wave == 0) {
        double tot = 0.0, tot2 = 0.0;
        for (int w = 0; w < kFinWaves; ++w) {
            tot += part[w][lane];
            tot2 += part2[w][lane];
        }
        if (pots) {
            if (in) gmem(fd.scf_sum)[col] = tot;
        } else {
            (void)column_epilogue<T>(fd, bins, jb.col0, f, tot, tot2, yt0, sg, Yj, lane);
        }
    }
    // the last job of this fit ends the step; in observe mode the same
    // hand-over runs on a separate counter and changes no state
    const uint32_t n_part = pot_mode ? (uint32_t)fd.n_pot_jobs
                                     : (cells_mode ? 0u : (uint32_t)fd.n_bin_jobs) +
                                           (f.refresh ? (uint32_t)fd.n_cell_jobs : 0u) +
                                           (f.pot ? (uint32_t)fd.n_pot_jobs : 0u);
    uint32_t* ticket = observe ? &st->mticket : &st->ticket;
    __syncthreads();
    if (threadIdx.x == 0) {
        // release of this job's results (wave 0 wrote them) with the count;
        // acquire of the others' for the last job, passed on to its block by
        // the barrier below
        const uint32_t prev =
            __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = (prev == n_part - 1) ? 1 : 0;
    }
    __syncthreads();
    if (!last) return;
    // a refresh with smoothing: the whole block smooths the prior grid
    if (fd.smooth && f.refresh)
    {
        // each n_E x n_x grid alone: the first, then the L_z < 0 half if split
        smooth_priors<T>(fd, 0, sgrid[0], sgrid[1], stab[0], stab[1], &part[0][0], &sidx, &smean);
        if (fd.C > fd.cell_half) {
            __syncthreads();
            smooth_priors<T>(fd, fd.cell_half, sgrid[0], sgrid[1], stab[0], stab[1], &part[0][0],
                             &sidx, &smean);
        }
    }
    // the node table of the self-consistent potential from the new sums
    if (SCF && f.pot) build_scf_table(fd);
    if (wave != 0) return;
    const double chi2 = (cells_mode || pot_mode)
                            ? 0.0
                            : chi2_of_parts(static_cast<const double*>(fd.chi2_part), fd.n_bin_jobs, lane);
    if (lane != 0) return;
    *ticket = 0u;
    if (observe || pot_mode) return;
    end_step(fd, gst, f, ss, chi2);
}

// the jobs of the fits of a table (batches)
template <typename T, bool SCF>
__global__ __launch_bounds__(kFinThreads) void k_finalize(const FitDev* __restrict__ fits,
                                                         const FinJob* __restrict__ jobs,
                                                         int32_t mode) {
    const FinJob jb = jobs[blockIdx.x];
    finalize_job<T, SCF>(fits[jb.fit], jb, mode);
}

// one fit, its description passed by value: block b < n_bin_jobs takes bin
// columns, then n_cell_jobs blocks cell columns, then n_pot_jobs blocks the
// columns of the self-consistent potential, over n_rows tile rows
template <typename T, bool SCF>
__global__ __launch_bounds__(kFinThreads) void k_finalize1(const FitDev fd, int32_t n_rows,
                                                          int32_t mode) {
    const int b = blockIdx.x;
    const int nb = fd.n_bin_jobs, nc = fd.n_cell_jobs;
    const int kind = b < nb ? 0 : (b < nb + nc ? 1 : 2);
    const int base = kind == 0 ? 0 : (kind == 1 ? nb : nb + nc);
    const FinJob jb{0, kind, (b - base) * kFinCols, n_rows};
    finalize_job<T, SCF>(fd, jb, mode);
}


// ------------------------------------------------------------- assign ------
template <typename T>
__global__ __launch_bounds__(256) void k_assign(const FitDev* __restrict__ fits,
                                                const Tile* __restrict__ tiles) {
    const Tile tl = tiles[blockIdx.x];
    const FitDev& fd = fits[tl.fit];
    const G<T> UH = gmem<T>(fd.uh);
    const G<const uint16_t> CI = gmem<const uint16_t>(fd.cidx);
    const G<const T> ucell = gmem<const T>(fd.ucell);
    const int C = fd.C;
    for (int64_t i = tl.begin + threadIdx.x; i < tl.end; i += 256)
        UH[i] = ucell[min((int)CI[i], C - 1)];
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // every tile of this launch belongs to one fit; the flag is consumed
        // by this launch as a whole and only read by later launches
        fd.st->assign_pending = 0;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_weights(const T* __restrict__ u, T* __restrict__ w,
                                                 int64_t n, double scale) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) w[i] = (T)((double)u[i] * scale);
}

__global__ void k_poke(FitState* st, int32_t steps_left, int32_t correct) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (steps_left >= 0) st->steps_left = steps_left;
        if (correct >= 0) st->correct = correct;
    }
}

__global__ void k_gather(const FitDev* __restrict__ fits, int n, int32_t* __restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        const FitState* st = fits[i].st;
        out[2 * i] = st->steps_left;
        out[2 * i + 1] = st->error;
    }
}

// Residuals, force table and chi^2 from the current ytilde (new targets).
template <typename T>
__global__ __launch_bounds__(256) void k_residuals(const FitDev* __restrict__ fits) {
    __shared__ double red[256];
    const FitDev& fd = fits[0];
    double d2 = 0.0;
    for (int j = threadIdx.x; j < fd.J; j += 256) {
        const double s = fd.sigma[j];
        const double d = (fd.ytil[j] - fd.Y[j]) / s;
        fd.delta[j] = d;
        static_cast<T*>(fd.rp)[j] = (T)(fd.foc_chi * d / s);
        d2 += d * d;
    }
    red[threadIdx.x] = d2;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        fd.st->chi2 = red[0];
        if (!isfinite(red[0])) fd.st->error |= 1;
    }
}

// one != nullptr: k_step1 over that fit (host copy passed by value), else
// k_step over the tables

}  // namespace

static hipError_t launch_step_any(bool f64, bool acc64, int block, int kin, const FitDev* fits,
                           const Tile* tiles, const FitDev* one, int n_tiles, size_t lds,
                           int32_t mode, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    if (f64) return launch_step_f64(256, kin, fits, tiles, one, n_tiles, lds, mode, s);
    if (acc64) return launch_step_f32d(block, kin, fits, tiles, one, n_tiles, lds, mode, s);
    return launch_step_f32f(block, kin, fits, tiles, one, n_tiles, lds, mode, s);
}


size_t step_lds_bytes(bool f64, bool acc64, int J, int n_r, int n_R, int n_v, int kpriv, int C,
                      int scf_nr, int scf_lmax) {
    (void)acc64;  // FP64 sums and FP32 sum + compensation both take 8 bytes per bin copy
    const size_t sz = f64 ? 8 : 4;
    const size_t bins = (size_t)J * (size_t)kpriv * 8 + (size_t)C * 8 + (size_t)((C + 1) & ~1) * 4;
    const size_t tabs = ((size_t)J + 2 * (size_t)(n_r + 1) + (size_t)(n_R + 1) + (size_t)(n_v + 1) +
                         2 * (size_t)n_R) * sz;
    const size_t scf = scf_nr > 0 ? scf_lds_bytes(scf_nr, scf_lmax, sz) : 0;
    return ((bins + tabs + scf + 15) / 16) * 16;
}

// Private bin copies: as many as fit in 48 KiB of LDS, at most 8.
int private_copies(bool f64, int J) {
    (void)f64;
    const size_t per = (size_t)J * 8;
    int k = 8;
    while (k > 1 && per * (size_t)k > 48 * 1024) k >>= 1;
    return k;
}

int kin_class(int kin, int gh_nmax, int dens, bool scf) {
    const int alm = (dens == 1 ? kKinAlm : 0) | (scf ? kKinScf : 0);
    switch (kin) {
        case 0: return alm | kKinNone;
        case 1: return alm | kKinV2;
        case 2: return alm | (gh_nmax == 4 ? kKinGH4 : kKinGHN);
        case 3: return alm | kKinLOSVD;
        default: return -1;
    }
}

hipError_t launch_step(bool f64, bool acc64, int block, int kin, const FitDev* fits,
                       const Tile* tiles, int n_tiles, size_t lds, int32_t mode, hipStream_t s) {
    return launch_step_any(f64, acc64, block, kin, fits, tiles, nullptr, n_tiles, lds, mode, s);
}

hipError_t launch_step1(bool f64, bool acc64, int block, int kin, const FitDev& fd, int n_tiles,
                        size_t lds, int32_t mode, hipStream_t s) {
    return launch_step_any(f64, acc64, block, kin, nullptr, nullptr, &fd, n_tiles, lds, mode, s);
}

hipError_t launch_finalize(bool f64, const FitDev* fits, int n_fits, const FinJob* jobs,
                           int n_jobs, int32_t mode, hipStream_t s, bool scf) {
    if (n_jobs <= 0) return hipSuccess;
    if (f64 && scf)
        hipLaunchKernelGGL((k_finalize<double, true>), dim3(n_jobs), dim3(kFinThreads), 0, s, fits,
                           jobs, mode);
    else if (f64)
        hipLaunchKernelGGL((k_finalize<double, false>), dim3(n_jobs), dim3(kFinThreads), 0, s,
                           fits, jobs, mode);
    else if (scf)
        hipLaunchKernelGGL((k_finalize<float, true>), dim3(n_jobs), dim3(kFinThreads), 0, s, fits,
                           jobs, mode);
    else
        hipLaunchKernelGGL((k_finalize<float, false>), dim3(n_jobs), dim3(kFinThreads), 0, s,
                           fits, jobs, mode);
    (void)n_fits;
    return hipGetLastError();
}

bool kin_scf(int kin) { return (kin & kKinScf) != 0; }

hipError_t launch_finalize1(bool f64, const FitDev& fd, int n_rows, int32_t mode, hipStream_t s) {
    const int n_jobs = fd.n_bin_jobs + fd.n_cell_jobs + fd.n_pot_jobs;
    if (n_jobs <= 0) return hipSuccess;
    const bool scf = fd.scf_nr > 0;
    if (f64 && scf)
        hipLaunchKernelGGL((k_finalize1<double, true>), dim3(n_jobs), dim3(kFinThreads), 0, s, fd,
                           n_rows, mode);
    else if (f64)
        hipLaunchKernelGGL((k_finalize1<double, false>), dim3(n_jobs), dim3(kFinThreads), 0, s, fd,
                           n_rows, mode);
    else if (scf)
        hipLaunchKernelGGL((k_finalize1<float, true>), dim3(n_jobs), dim3(kFinThreads), 0, s, fd,
                           n_rows, mode);
    else
        hipLaunchKernelGGL((k_finalize1<float, false>), dim3(n_jobs), dim3(kFinThreads), 0, s, fd,
                           n_rows, mode);
    return hipGetLastError();
}

hipError_t launch_assign(bool f64, const FitDev* fits, const Tile* tiles, int n_tiles,
                         hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL(k_assign<double>, dim3(n_tiles), dim3(256), 0, s, fits, tiles);
    else
        hipLaunchKernelGGL(k_assign<float>, dim3(n_tiles), dim3(256), 0, s, fits, tiles);
    return hipGetLastError();
}

hipError_t launch_weights(bool f64, const void* u, void* w, int64_t n, double scale,
                          hipStream_t s) {
    const int64_t blocks = (n + 255) / 256;
    if (blocks <= 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL(k_weights<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                           static_cast<const double*>(u), static_cast<double*>(w), n, scale);
    else
        hipLaunchKernelGGL(k_weights<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                           static_cast<const float*>(u), static_cast<float*>(w), n, scale);
    return hipGetLastError();
}

hipError_t launch_poke(FitState* st, int32_t steps_left, int32_t correct, hipStream_t s) {
    hipLaunchKernelGGL(k_poke, dim3(1), dim3(64), 0, s, st, steps_left, correct);
    return hipGetLastError();
}

hipError_t launch_gather(const FitDev* fits, int n, int32_t* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3((n + 255) / 256), dim3(256), 0, s, fits, n, out);
    return hipGetLastError();
}

hipError_t launch_residuals(bool f64, const FitDev* fit, hipStream_t s) {
    if (f64)
        hipLaunchKernelGGL(k_residuals<double>, dim3(1), dim3(256), 0, s, fit);
    else
        hipLaunchKernelGGL(k_residuals<float>, dim3(1), dim3(256), 0, s, fit);
    return hipGetLastError();
}

}  // namespace m2m

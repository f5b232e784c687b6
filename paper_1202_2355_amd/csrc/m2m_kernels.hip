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
// of lambda, summed by one wave over the n eigenvalues (in g2) and the
// transformed data (in wh); 1 / (1 + t) is a hardware reciprocal refined by two Newton
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
// with the GCV-chosen lambda (Sec. 2.3.2, eq. smooth_grid) by the block that
// ends a refresh step. The penalty P (finite-difference second derivatives
// where their stencils fit the grid) has the eigendecomposition
// P = Q diag(g) Q^T that the host computed per grid shape (fd.sm_basis): Q is
// the parity basis of the two axis reflections (even/odd pairs of cells)
// times the eigenvectors of four parity blocks. With w^ = Q^T w0 the
// smoother is the filter 1/(1 + lambda g), and with t = lambda g
//   |w0 - A w0|^2 = sum (t/(1+t))^2 w^^2,  1 - tr(A)/n = sum t/(1+t) / n.
// The log10(lambda) search: steps of 0.25 from sm_plo (sm_k1 points), then
// 65 points over the two steps around the best, then 65 points over the two
// sub-steps around the best (first minimum on ties). Smoothed priors are
// floored at 1e-3 of the mean of the data.
// LDS: the folded grid / eigenvalues in sa, the transformed data in sb
// (kSmoothMaxCells doubles each), buf (scores and lambdas of a search stage).

// Parity blocks of an axis of n cells: (n+1)/2 even and n/2 odd vectors.
// Coefficient of cell k in vector i of parity p (cells i and n-1-i).
__device__ __forceinline__ double fold_coef(int n, int p, int i, int k) {
    const int i2 = n - 1 - i;
    if (i == i2) return (p == 0 && k == i) ? 1.0 : 0.0;
    const double s = 0.70710678118654752440;
    if (k == i) return s;
    if (k == i2) return p == 0 ? s : -s;
    return 0.0;
}

// sum_k A[k stride] x[k] over k < m (A in global memory, x in LDS) with
// kDotDepth loads in flight per thread: one block reads the smoothing basis
// alone, so it is bound by how many of its loads are outstanding, not by
// bandwidth; four partial sums, combined at the end.
constexpr int kDotDepth = 16;
__device__ __forceinline__ double dot_global(G<const double> A, size_t stride, const double* x,
                                             int m) {
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    int k = 0;
    for (; k + kDotDepth <= m; k += kDotDepth) {
        double q[kDotDepth];
#pragma unroll
        for (int u = 0; u < kDotDepth; ++u) q[u] = A[(size_t)(k + u) * stride];
#pragma unroll
        for (int u = 0; u < kDotDepth; u += 4) {
            acc0 = fma(q[u], x[k + u], acc0);
            acc1 = fma(q[u + 1], x[k + u + 1], acc1);
            acc2 = fma(q[u + 2], x[k + u + 2], acc2);
            acc3 = fma(q[u + 3], x[k + u + 3], acc3);
        }
    }
    for (; k < m; ++k) acc0 = fma(A[(size_t)k * stride], x[k], acc0);
    return (acc0 + acc1) + (acc2 + acc3);
}

// The four parity blocks of an n_E x n_x grid: block b = 2 pE + pX holds
// mE(pE) mX(pX) folded coefficients from off(b) and its eigenvectors from
// qoff(b) in the basis (scalars and selects, no indexed arrays, so that
// nothing goes to scratch memory).
struct SmBlocks {
    int mE0, mE1, mX0, mX1;
    int o1, o2, o3, o4;  // off(1..4); off(0) = 0
    int q0, q1, q2, q3;  // qoff(0..3)
    __device__ int mE(int p) const { return p ? mE1 : mE0; }
    __device__ int mX(int p) const { return p ? mX1 : mX0; }
    __device__ int off(int b) const {
        return b == 0 ? 0 : (b == 1 ? o1 : (b == 2 ? o2 : (b == 3 ? o3 : o4)));
    }
    __device__ int qoff(int b) const { return b == 0 ? q0 : (b == 1 ? q1 : (b == 2 ? q2 : q3)); }
    // the block of folded index c (0 <= c < n_E n_x)
    __device__ int block_of(int c) const { return c < o1 ? 0 : (c < o2 ? 1 : (c < o3 ? 2 : 3)); }
};

__device__ __forceinline__ SmBlocks sm_blocks(int nE, int nx) {
    SmBlocks B;
    B.mE0 = (nE + 1) / 2;
    B.mE1 = nE / 2;
    B.mX0 = (nx + 1) / 2;
    B.mX1 = nx / 2;
    const int m0 = B.mE0 * B.mX0, m1 = B.mE0 * B.mX1, m2 = B.mE1 * B.mX0, m3 = B.mE1 * B.mX1;
    B.o1 = m0;
    B.o2 = m0 + m1;
    B.o3 = m0 + m1 + m2;
    B.o4 = m0 + m1 + m2 + m3;
    B.q0 = nE * nx;
    B.q1 = B.q0 + m0 * m0;
    B.q2 = B.q1 + m1 * m1;
    B.q3 = B.q2 + m2 * m2;
    return B;
}

template <typename T>
__device__ __forceinline__ void smooth_priors(const FitDev& fd, int base, double* sa, double* sb,
                                              double* buf, int* sidx, double* smean) {
    static_assert(2 * kSmoothMaxPoints <= kFinWaves * kFinCols, "GCV scores and lambdas in buf");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nE = fd.n_E, nx = fd.n_x, n = nE * nx;
    const G<const double> w0 = gmem<const double>(fd.cdata) + base;
    const G<double> gp = gmem(fd.gprior) + base;
    const G<T> uc = gmem<T>(fd.ucell) + base;
    const G<const double> basis = gmem<const double>(fd.sm_basis);
    if (n < 2) {
        if (tid == 0) {
            gp[0] = w0[0];
            uc[0] = (T)w0[0];
        }
        return;
    }
    const SmBlocks B = sm_blocks(nE, nx);
    if (wave == 0) {
        double sm = 0.0;
        for (int c = lane; c < n; c += 64) sm += w0[c];
        for (int off = 32; off >= 1; off >>= 1) sm += __shfl_xor(sm, off, 64);
        if (lane == 0) *smean = sm / n;
    }
    // fold: the coefficient of each parity-basis vector, from its (up to)
    // four cells (k, l) with k in {i, nE-1-i}, l in {j, nx-1-j}
    for (int c = tid; c < n; c += kFinThreads) {
        const int b = B.block_of(c), pE = b >> 1, pX = b & 1;
        const int r = c - B.off(b), i = r / B.mX(pX), j = r - i * B.mX(pX);
        const int k1 = nE - 1 - i, l1 = nx - 1 - j;
        const double ce0 = fold_coef(nE, pE, i, i), ce1 = k1 != i ? fold_coef(nE, pE, i, k1) : 0.0;
        const double cx0 = fold_coef(nx, pX, j, j), cx1 = l1 != j ? fold_coef(nx, pX, j, l1) : 0.0;
        double v = ce0 * cx0 * w0[i * nx + j];
        if (l1 != j) v += ce0 * cx1 * w0[i * nx + l1];
        if (k1 != i) {
            v += ce1 * cx0 * w0[k1 * nx + j];
            if (l1 != j) v += ce1 * cx1 * w0[k1 * nx + l1];
        }
        sa[c] = v;
    }
    __syncthreads();
    // w^ = Q_b^T (folded data), one output per thread: Q_b[r][o] over r,
    // consecutive o in consecutive lanes
    for (int c = tid; c < n; c += kFinThreads) {
        const int b = B.block_of(c), m = B.off(b + 1) - B.off(b);
        const int o = c - B.off(b);
        sb[c] = dot_global(basis + B.qoff(b) + o, (size_t)m, sa + B.off(b), m);
    }
    __syncthreads();
    for (int c = tid; c < n; c += kFinThreads) sa[c] = basis[c];  // eigenvalues
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
    // filter into sa, then back: folded coefficients Q_b (filtered w^), one
    // row per thread, into sb
    for (int c = tid; c < n; c += kFinThreads) sa[c] = sb[c] / (1.0 + lam * sa[c]);
    __syncthreads();
    for (int c = tid; c < n; c += kFinThreads) {
        const int bb = B.block_of(c), m = B.off(bb + 1) - B.off(bb);
        const int r = c - B.off(bb);
        sb[c] = dot_global(basis + B.qoff(bb) + (size_t)r * m, 1, sa + B.off(bb), m);
    }
    __syncthreads();
    // unfold: cell (k, l) from the vectors of both parities that touch it
    const double floor_v = 1e-3 * (*smean);
    for (int o = tid; o < n; o += kFinThreads) {
        const int k = o / nx, l = o - k * nx;
        const int i = min(k, nE - 1 - k), j = min(l, nx - 1 - l);
        double v = 0.0;
        for (int pE = 0; pE < 2; ++pE) {
            if (i >= B.mE(pE)) continue;
            const double ce = fold_coef(nE, pE, i, k);
            if (ce == 0.0) continue;
            for (int pX = 0; pX < 2; ++pX) {
                if (j >= B.mX(pX)) continue;
                const double cx = fold_coef(nx, pX, j, l);
                if (cx == 0.0) continue;
                const int bb = 2 * pE + pX;
                v += ce * cx * sb[B.off(bb) + i * B.mX(pX) + j];
            }
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

// LDS grids of the prior smoothing, only in the finalize variant that has it
template <bool SMOOTH>
struct SmoothLds {
    double g[2][kSmoothMaxCells];
};
template <>
struct SmoothLds<false> {};

// SCF: the fit has the self-consistent potential (its potential jobs and the
// node table are compiled in only then); SMOOTH: some fit of the launch
// smooths its prior grid.
//
// Every launched job of a fit takes one ticket, also the jobs with nothing
// to do in this launch (cell columns on steps without a refresh, potential
// columns on steps without a rebuild, observable columns in the modes that
// reduce only cells or the potential). The job that takes the last ticket
// ends the step and rewrites the fit's counters, so it can only do so once
// every job has read them: a job that read the counters after the end of
// the step would see the next step's schedule.
template <typename T, bool SCF, bool SMOOTH>
__device__ __forceinline__ void finalize_job(const FitDev& fd, const FinJob& jb, int32_t mode) {
    __shared__ double part[kFinWaves][kFinCols];
    __shared__ double part2[kFinWaves][kFinCols];
    __shared__ int last, sidx;
    __shared__ double smean;
    __shared__ SmoothLds<SMOOTH> sl;
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
    // an idle fit: every job of it reads steps_left <= 0 (no job of this
    // launch ends its step), and none takes a ticket
    if (step && ss.steps_left <= 0) return;
    const Flags f = flags_of<SCF>(fd, ss, mode);
    // this job's work in this launch
    const bool work = bins ? !(cells_mode || pot_mode) : (jb.kind == 1 ? f.refresh : (pots && f.pot));
    if (work) {
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
    }
    // the last job of this fit ends the step; in observe mode the same
    // hand-over runs on a separate counter and changes no state
    const uint32_t n_part = (uint32_t)(fd.n_bin_jobs + fd.n_cell_jobs + fd.n_pot_jobs);
    uint32_t* ticket = observe ? &st->mticket : &st->ticket;
    __syncthreads();
    if (threadIdx.x == 0) {
        // a job with results: release of them (wave 0 wrote them) with the
        // count; acquire of the others' for the last job, passed on to its
        // block by the barrier below. A job without results only counts
        // itself: its reads of the counters have completed, as their values
        // decided the branch that led here, so a relaxed add suffices (an
        // agent-scope release would write back the whole L2 of its XCD); if
        // it is the last, it acquires the others' results by a fence.
        uint32_t prev;
        if (work) {
            prev = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            prev = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (prev == n_part - 1) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        last = (prev == n_part - 1) ? 1 : 0;
    }
    __syncthreads();
    if (!last) return;
    // a refresh with smoothing: the whole block smooths the prior grid, each
    // n_E x n_x grid alone (the first, then the L_z < 0 half if split)
    if constexpr (SMOOTH) {
        if (fd.smooth && f.refresh) {
            smooth_priors<T>(fd, 0, sl.g[0], sl.g[1], &part[0][0], &sidx, &smean);
            if (fd.C > fd.cell_half) {
                __syncthreads();
                smooth_priors<T>(fd, fd.cell_half, sl.g[0], sl.g[1], &part[0][0], &sidx, &smean);
            }
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

// One block reduces every column of one fit and ends its step (batches of
// fits with few tile rows): the observable columns in chunks of kFinCols
// (each chunk summed over the rows exactly as one column job sums them,
// then its epilogue and its chi^2 part), on refresh steps the cell columns,
// on rebuild steps the potential columns, then the smoothing, the node table,
// chi^2 from the parts in chunk order and the step counters. Nothing else
// reads or writes the fit's counters during the launch, so no ticket is
// taken. The results equal those of the column jobs bit for bit.
constexpr int kMaxChunks = 16384 / kFinCols;
constexpr int kFitChunks = 4;  // column chunks summed together by the whole-fit finalize

// Row group `wave` (of NW) of nb <= kFitChunks chunks of kFinCols columns
// from column base + c0 (columns c < ncols of the section): for each column
// the sum of rows wave, wave + NW, ... in row order (with counts from column
// + C for cells); four rows of every chunk in flight.
template <int NW>
__device__ __forceinline__ void chunk_sums(const FitDev& fd, int base, int c0, int ncols, int nb,
                                           bool counts, int n_rows, int wave, int lane,
                                           double* acc, double* acc2) {
    const size_t stride = (size_t)fd.row_len;
    const G<const double> P = gmem<const double>(fd.partials) + base;
    bool ok[kFitChunks];
#pragma unroll
    for (int k = 0; k < kFitChunks; ++k) {
        acc[k] = acc2[k] = 0.0;
        ok[k] = k < nb && c0 + k * kFinCols + lane < ncols;
    }
    for (int t0 = wave; t0 < n_rows; t0 += 4 * NW) {
        double v[4][kFitChunks], w[4][kFitChunks];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int t = t0 + u * NW;
#pragma unroll
            for (int k = 0; k < kFitChunks; ++k) {
                const size_t at = (size_t)t * stride + c0 + k * kFinCols + lane;
                v[u][k] = (t < n_rows && ok[k]) ? P[at] : 0.0;
                w[u][k] = (counts && t < n_rows && ok[k]) ? P[at + fd.C] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < kFitChunks; ++k) {
                acc[k] += v[u][k];
                acc2[k] += w[u][k];
            }
    }
}

// NW waves (row groups); the smoothing needs a block of kFinWaves waves.
template <typename T, bool SCF, bool SMOOTH, int NW>
__device__ __forceinline__ void finalize_fit(const FitDev& fd, int n_rows, int32_t mode) {
    static_assert(!SMOOTH || NW == kFinWaves, "prior smoothing needs kFinWaves waves");
    __shared__ double part[NW][kFinCols];
    __shared__ double part2[NW][kFinCols];
    __shared__ double chi2p[kMaxChunks];
    __shared__ int sidx;
    __shared__ double smean;
    __shared__ SmoothLds<SMOOTH> sl;
    const G<FitState> gst = gmem(fd.st);
    const bool cells_mode = (mode & kModeCells) != 0;
    const bool observe = (mode & kModeObserve) != 0;
    const bool pot_mode = SCF && (mode & kModePot) != 0;
    const bool step = (mode & kModeStep) != 0;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const Snap ss = snap_of(gst);
    if (step && ss.steps_left <= 0) return;  // uniform: the fit is idle
    const Flags f = flags_of<SCF>(fd, ss, mode);
    const int nbj = fd.n_bin_jobs;
    // observable columns, up to kFitChunks chunks of kFinCols at a time: their
    // row loads (and wave 0's epilogue inputs) are all issued before any sum
    if (!cells_mode && !pot_mode)
        for (int b0 = 0; b0 < nbj; b0 += kFitChunks) {
            const int nb = min(kFitChunks, nbj - b0);
            double acc[kFitChunks], acc2[kFitChunks], yt0[kFitChunks], sg[kFitChunks], Yj[kFitChunks];
#pragma unroll
            for (int k = 0; k < kFitChunks; ++k) {
                acc[k] = acc2[k] = yt0[k] = Yj[k] = 0.0;
                sg[k] = 1.0;
                const int col = (b0 + k) * kFinCols + lane;
                if (k < nb && col < fd.J && wave == 0 && !observe) {
                    yt0[k] = gmem(fd.ytil)[col];
                    sg[k] = gmem(fd.sigma)[col];
                    Yj[k] = gmem(fd.Y)[col];
                }
            }
            chunk_sums<NW>(fd, 0, b0 * kFinCols, fd.J, nb, false, n_rows, wave, lane, acc, acc2);
            for (int k = 0; k < nb; ++k) {
                part[wave][lane] = acc[k];
                __syncthreads();
                if (wave == 0) {
                    double tot = 0.0;
                    for (int w = 0; w < NW; ++w) tot += part[w][lane];
                    const double d2 = column_epilogue<T>(fd, true, (b0 + k) * kFinCols, f, tot, 0.0,
                                                         yt0[k], sg[k], Yj[k], lane);
                    if (lane == 0) chi2p[b0 + k] = d2;
                }
                __syncthreads();
            }
        }
    // cell columns on refresh steps (sums and counts)
    if (f.refresh)
        for (int b0 = 0; b0 < fd.n_cell_jobs; b0 += kFitChunks) {
            const int nb = min(kFitChunks, fd.n_cell_jobs - b0);
            double acc[kFitChunks], acc2[kFitChunks];
            chunk_sums<NW>(fd, fd.J, b0 * kFinCols, fd.C, nb, true, n_rows, wave, lane, acc, acc2);
            for (int k = 0; k < nb; ++k) {
                part[wave][lane] = acc[k];
                part2[wave][lane] = acc2[k];
                __syncthreads();
                if (wave == 0) {
                    double tot = 0.0, tot2 = 0.0;
                    for (int w = 0; w < NW; ++w) {
                        tot += part[w][lane];
                        tot2 += part2[w][lane];
                    }
                    (void)column_epilogue<T>(fd, false, (b0 + k) * kFinCols, f, tot, tot2, 0.0, 1.0,
                                             0.0, lane);
                }
                __syncthreads();
            }
        }
    // potential columns on rebuild steps
    if (SCF && f.pot)
        for (int b0 = 0; b0 < fd.n_pot_jobs; b0 += kFitChunks) {
            const int nb = min(kFitChunks, fd.n_pot_jobs - b0);
            double acc[kFitChunks], acc2[kFitChunks];
            chunk_sums<NW>(fd, fd.scf_col0, b0 * kFinCols, fd.scf_P, nb, false, n_rows, wave, lane, acc,
                       acc2);
            for (int k = 0; k < nb; ++k) {
                const int col = (b0 + k) * kFinCols + lane;
                part[wave][lane] = acc[k];
                __syncthreads();
                if (wave == 0 && col < fd.scf_P) {
                    double tot = 0.0;
                    for (int w = 0; w < NW; ++w) tot += part[w][lane];
                    gmem(fd.scf_sum)[col] = tot;
                }
                __syncthreads();
            }
        }
    // the prior smoothing, then the node table (the block's own writes above
    // are ordered before them by the barriers)
    if constexpr (SMOOTH) {
        if (fd.smooth && f.refresh) {
            smooth_priors<T>(fd, 0, sl.g[0], sl.g[1], &part[0][0], &sidx, &smean);
            if (fd.C > fd.cell_half) {
                __syncthreads();
                smooth_priors<T>(fd, fd.cell_half, sl.g[0], sl.g[1], &part[0][0], &sidx, &smean);
            }
        }
    }
    if (SCF && f.pot) build_scf_table(fd);
    if (wave != 0) return;
    const double chi2 = (cells_mode || pot_mode) ? 0.0 : chi2_of_parts(chi2p, nbj, lane);
    if (lane != 0 || observe || pot_mode) return;
    end_step(fd, gst, f, ss, chi2);
}

// the column jobs of the fits of a table (batches of fits with many rows)
template <typename T, bool SCF, bool SMOOTH>
__global__ __launch_bounds__(kFinThreads) void k_finalize(const FitDev* __restrict__ fits,
                                                         const FinJob* __restrict__ jobs,
                                                         int32_t mode) {
    const FinJob jb = jobs[blockIdx.x];
    finalize_job<T, SCF, SMOOTH>(fits[jb.fit], jb, mode);
}

// one block of NW waves per fit of a table, each reducing every column of
// its fit (batches of fits with few rows); blocks of one wave per SIMD, so
// that they find room beside the step kernel of another group of the batch
template <typename T, bool SCF, bool SMOOTH, int NW>
__global__ __launch_bounds__(NW * 64) void k_finalize_fits(const FitDev* __restrict__ fits,
                                                          const FinJob* __restrict__ jobs,
                                                          int32_t mode) {
    const FinJob jb = jobs[blockIdx.x];
    finalize_fit<T, SCF, SMOOTH, NW>(fits[jb.fit], jb.n_tiles, mode);
}

// one fit, its description passed by value: block b < n_bin_jobs takes bin
// columns, then n_cell_jobs blocks cell columns, then n_pot_jobs blocks the
// columns of the self-consistent potential, over n_rows tile rows
template <typename T, bool SCF, bool SMOOTH>
__global__ __launch_bounds__(kFinThreads) void k_finalize1(const FitDev fd, int32_t n_rows,
                                                          int32_t mode) {
    const int b = blockIdx.x;
    const int nb = fd.n_bin_jobs, nc = fd.n_cell_jobs;
    const int kind = b < nb ? 0 : (b < nb + nc ? 1 : 2);
    const int base = kind == 0 ? 0 : (kind == 1 ? nb : nb + nc);
    const FinJob jb{0, kind, (b - base) * kFinCols, n_rows};
    finalize_job<T, SCF, SMOOTH>(fd, jb, mode);
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

namespace {
constexpr int kFitWaves = 4;  // waves of a whole-fit finalize block without smoothing

template <bool SCF, bool SMOOTH>
hipError_t launch_fin_t(bool f64, const FitDev* fits, const FinJob* jobs, const FitDev* one,
                        int n_blocks, int n_rows, int32_t mode, hipStream_t s, bool whole) {
    if (one) {
        if (f64)
            hipLaunchKernelGGL((k_finalize1<double, SCF, SMOOTH>), dim3(n_blocks), dim3(kFinThreads), 0,
                               s, *one, n_rows, mode);
        else
            hipLaunchKernelGGL((k_finalize1<float, SCF, SMOOTH>), dim3(n_blocks), dim3(kFinThreads), 0,
                               s, *one, n_rows, mode);
    } else if (whole) {
        constexpr int NW = SMOOTH ? kFinWaves : kFitWaves;
        if (f64)
            hipLaunchKernelGGL((k_finalize_fits<double, SCF, SMOOTH, NW>), dim3(n_blocks),
                               dim3(NW * 64), 0, s, fits, jobs, mode);
        else
            hipLaunchKernelGGL((k_finalize_fits<float, SCF, SMOOTH, NW>), dim3(n_blocks),
                               dim3(NW * 64), 0, s, fits, jobs, mode);
    } else {
        if (f64)
            hipLaunchKernelGGL((k_finalize<double, SCF, SMOOTH>), dim3(n_blocks), dim3(kFinThreads), 0,
                               s, fits, jobs, mode);
        else
            hipLaunchKernelGGL((k_finalize<float, SCF, SMOOTH>), dim3(n_blocks), dim3(kFinThreads), 0,
                               s, fits, jobs, mode);
    }
    return hipGetLastError();
}

hipError_t launch_fin_any(bool f64, bool scf, bool smooth, const FitDev* fits, const FinJob* jobs,
                          const FitDev* one, int n_blocks, int n_rows, int32_t mode, hipStream_t s,
                          bool whole) {
    if (n_blocks <= 0) return hipSuccess;
    if (scf && smooth)
        return launch_fin_t<true, true>(f64, fits, jobs, one, n_blocks, n_rows, mode, s, whole);
    if (scf) return launch_fin_t<true, false>(f64, fits, jobs, one, n_blocks, n_rows, mode, s, whole);
    if (smooth) return launch_fin_t<false, true>(f64, fits, jobs, one, n_blocks, n_rows, mode, s, whole);
    return launch_fin_t<false, false>(f64, fits, jobs, one, n_blocks, n_rows, mode, s, whole);
}
}  // namespace

hipError_t launch_finalize(bool f64, const FitDev* fits, int n_fits, const FinJob* jobs,
                           int n_jobs, int32_t mode, hipStream_t s, bool scf, bool smooth,
                           bool whole) {
    (void)n_fits;
    return launch_fin_any(f64, scf, smooth, fits, jobs, nullptr, n_jobs, 0, mode, s, whole);
}

bool kin_scf(int kin) { return (kin & kKinScf) != 0; }

hipError_t launch_finalize1(bool f64, const FitDev& fd, int n_rows, int32_t mode, hipStream_t s) {
    const int n_jobs = fd.n_bin_jobs + fd.n_cell_jobs + fd.n_pot_jobs;
    return launch_fin_any(f64, fd.scf_nr > 0, fd.smooth != 0, nullptr, nullptr, &fd, n_jobs, n_rows,
                          mode, s, false);
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

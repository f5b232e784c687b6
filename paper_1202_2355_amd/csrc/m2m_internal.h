// Internal device-side structures shared by the HIP kernels (m2m_kernels.hip)
// and the host side of the C ABI (m2m_api.cpp). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace m2m {

constexpr int kMaxGH = 8;          // largest Gauss-Hermite order
constexpr int kMaxLOSVD = 256;     // largest LOSVD bin count
constexpr int kMaxLM = 8;          // largest degree l of the a_lm density observables
constexpr int kMaxCells = 4096;    // largest n_E * n_x
constexpr int kLcTable = 8192;     // entries of the ln r_c(ln zeta) table
constexpr int kFinCols = 64;       // columns (bins or cells) per finalize block
constexpr int kFinThreads = 1024;  // finalize block: 16 waves over the tiles
constexpr int kFinWaves = kFinThreads / 64;  // row groups of the fixed reduction order
constexpr int kSmoothMaxSide = 128;   // prior smoothing: at most this many cells per axis
constexpr int kSmoothMaxCells = 2048; // and per smoothed grid
constexpr int kSmoothMaxPoints = 256; // and at most this many first-stage search points
constexpr int kGcvSlots = 5;          // lambda points a wave scores in one pass over the cells
constexpr int kHistCap = 8192;     // chi^2 history ring per fit
constexpr int kSegAlign = 64;      // tile boundaries are multiples of 64 particles
constexpr int kMaxScfNodes = 64;   // largest node count of the self-consistent potential

// kernel launch modes (bit set)
enum : int32_t {
    kModeStep = 1,       // a full M2M step: (assign) FOC, push, deposit, (cells)
    kModeInit = 2,       // deposit the current state; finalize sets ytilde = y
    kModeObserve = 4,    // deposit the current state into obs_out only
    kModeCells = 8,      // accumulate the prior cells of the current state only
    kModeWriteThrough = 16,  // step: particle stores write through L2 (small fits)
    kModePot = 32,       // rebuild the self-consistent potential from the current state only
    kModeStream = 64,    // batch step: nontemporal particle loads and stores (large states)
    kModeInterleave = 128,  // one fit: tiles take interleaved chunks of particles (large states)
};

// Particle state up to this size is stepped with write-through stores: it
// stays in the memory-side cache, and no dirty particle lines are left in L2
// for the write-back at the end of the step kernel.
constexpr size_t kWriteThroughMax = size_t(64) << 20;

// The particle state of a batch launch above this size is streamed with
// nontemporal loads and stores (the batch step kernels of the lean kinds of
// observables, FP32 state): it does not fit the memory-side cache anyway, and with the
// hint on both the loads and the stores the 64-fit batch of 1.16 GB stepped
// 11 % faster; either hint alone gained nothing, and a state that stays in
// the cache (3.2e7 bytes) stepped 6 % slower with them.
constexpr size_t kStreamMin = size_t(128) << 20;

// The step kernel of one fit whose particle state exceeds kStreamMin takes
// its particles interleaved (kModeInterleave): chunks of one block's width,
// dealt to the tiles in turn, so that the blocks in flight read and write a
// narrow window of each array. At 8e6 particles (480 MB) the step kernel ran
// 10 % faster so; at 1e6 (in the memory-side cache) 2-4 % slower, and the
// 64-fit batch (many fits of about 24 tiles each) gained nothing.

// Dynamic per-fit state, device resident, written only by the kernels (and by
// the host between launches, on the fit's stream).
struct FitState {
    int64_t kstep;           // correction steps done (prior schedule)
    int64_t tstep;           // all steps done (chi^2 history index)
    int32_t steps_left;      // steps still to run; kernels skip the fit at 0
    int32_t correct;         // force of change on (1) or relaxation (0)
    int32_t assign_pending;  // fresh cell priors wait to be assigned
    int32_t error;           // bit 0: non-finite chi^2 seen
    uint32_t ticket;         // finalize: blocks done this launch
    uint32_t mticket;        // the same in observe mode
    double chi2;             // chi^2 after the last step
};

// Static per-fit description (device copy). Pointers are device addresses.
struct FitDev {
    // particle state (float or double, SoA)
    void *x, *y, *z, *vx, *vy, *vz, *u, *uh;
    int64_t n;
    // potential: Hernquist G M upsilon, a; NFW G M200 / f(c), r_s; Phi(0)
    double GMh, a, GMn, rs, phi0;
    // observables
    int32_t n_r, n_R, kin, nk, J, n_v, gh_nmax, C;
    int32_t jk0;             // index of the first kinematic observable
    int32_t l_max;           // a_lm degree; n_r then counts mesh intervals
    double lr0, lrs;         // radial bin guess: (log2(r^2) - lr0) * lrs
    double lR0, lRs;         // annulus bin guess
    double vmin, vidv;       // LOSVD bin guess: (v - vmin) * vidv
    void *redge2, *Redge2, *vedge, *Vp, *isp, *rp;  // tables in the state dtype
    void* rmesh;             // a_lm mesh radii (n_r + 1, state dtype)
    double *Y, *sigma, *yv, *ytil, *delta, *obs_out;
    double *partials;        // tile rows of row_len doubles
    int32_t row_len;         // J + 2 C (+ scf_P)
    int32_t kpriv;           // private copies of the in-tile bins (power of 2)
    int32_t smooth;          // thin-plate smoothing of the prior grid at refreshes
    int32_t n_bin_jobs;      // ceil(J / kFinCols)
    int32_t n_cell_jobs;     // ceil(C / kFinCols)
    int32_t entropy;
    // priors
    int32_t n_E, n_x, prior_every, pad1;
    double E_lo, E_hi, E_scale;  // E_scale = n_E / (E_hi - E_lo)
    // energy coordinate of the cells: (e - cell_e0) * cell_es with e = E, or
    // e = exp(E) (cell_flags bit 1); bit 0: particles with L_z < 0 take cell
    // cell_half + k n_x + l
    double cell_e0, cell_es;
    int32_t cell_flags, cell_half;
    void *ucell, *lctab;         // C values; kLcTable values of ln r_c(ln zeta)
    uint16_t *cidx;              // n values: cell of each particle at the last refresh
    // prior grid in FP64: cell data of the last refresh (means, or the
    // previous prior of empty cells) and the current priors
    double *cdata, *gprior;
    // smoothing: the log10(lambda) search range, the cell width along energy
    double sm_plo, sm_phi, sm_hE;
    int32_t sm_k1, pad3;         // points of the first search stage
    // eigenvalues and parity-block eigenvectors of the smoothing penalty
    // (smooth_basis below), FP64
    double* sm_basis;
    double lz0, ilz;             // ln zeta of entry 0, 1 / step in ln zeta
    double hv2, hr02, hiq2;      // logarithmic halo: v0^2 (0: none), r0^2, 1/q^2
    // step constants
    double dt, w0, foc_mu, foc_cs, foc_chi, q;  // foc_mu = eps dt mu, foc_chi = eps dt w0
    double *chi2_hist;
    double *chi2_part;           // one per bin job
    FitState *st;
    // self-consistent stellar potential (last, so that the fields before keep
    // their offsets in the kernel arguments) (scf_nr = 0: none): a multipole
    // expansion to degree scf_lmax with node values at scf_nr radii
    // log-spaced from scf_rho[0]; the tile rows carry its scf_P interval sums
    // from column scf_col0 (after the cell columns), reduced by n_pot_jobs
    // finalize jobs on the steps that rebuild it (every scf_every steps)
    int32_t scf_nr, scf_lmax, scf_every, scf_col0, scf_P, n_pot_jobs;
    double scf_ls0, scf_ih;      // ln rho_0, 1 / node spacing in ln r
    double scf_c;                // G upsilon M / N: Phi scale per unit weight u
    double *scf_rho;             // node radii (FP64)
    double *scf_sum;             // interval sums of the last rebuild (scf_P)
    double *scf_tab;             // nodes x (l, m): Phi_lm(rho_k), r dPhi_lm/dr there
};

// One tile: a contiguous particle range of one fit, owned by one block.
struct Tile {
    int32_t fit;     // index into the launch's fit table
    int32_t row;     // tile row in the fit's partials
    int64_t begin, end;
    int32_t n_rows;  // tiles of this fit in the launch
    int32_t pad;
};

// Tile t of count tiles over n particles (tile rows row0 + t of fit `fit`):
// boundaries at n t / count rounded down to a multiple of kSegAlign, the
// last tile ending at n. The host builds its tile tables with it, and the
// one-fit step kernel finds its own tile with it.
__host__ __device__ inline Tile tile_of(int64_t n, int t, int count, int fit, int row0) {
    int64_t b = n * t / count, e = n * (t + 1) / count;
    b = b / kSegAlign * kSegAlign;
    e = (t == count - 1) ? n : e / kSegAlign * kSegAlign;
    return Tile{fit, row0 + t, b, e, count, 0};
}

// One finalize block: kFinCols columns of one fit, or (kind kFinWholeFit)
// every column of one fit and the end of its step.
constexpr int32_t kFinWholeFit = 3;
struct FinJob {
    int32_t fit;
    int32_t kind;  // 0: observable columns, 1: cell columns, 2: potential columns, 3: all
    int32_t col0;
    int32_t n_tiles;  // rows of the fit to reduce
};

// ---- launchers (m2m_kernels.hip) ------------------------------------------
// kin: kinematic kind of every fit in the launch, from kin_class()
hipError_t launch_step(bool f64, bool acc64, int block, int kin, const FitDev* fits,
                       const Tile* tiles, int n_tiles, size_t lds_bytes, int32_t mode,
                       hipStream_t s);
// the column jobs of the fits of the table (n_fits of them)
// scf: the fits have the self-consistent potential (kin_scf of their kin class)
// smooth: some fit of the launch smooths its prior grid (the variant with the
// smoothing's LDS grids); whole: every job is a whole-fit job (one block per
// fit, the kernel with small blocks), else every job is a column job
hipError_t launch_finalize(bool f64, const FitDev* fits, int n_fits, const FinJob* jobs,
                           int n_jobs, int32_t mode, hipStream_t s, bool scf, bool smooth,
                           bool whole);
bool kin_scf(int kin);
// the step kernel of one particle-state / in-tile-sum type pair (one == nullptr:
// over the fit and tile tables, else over that one fit); m2m_step_*.hip
hipError_t launch_step_f64(int block, int kin, const FitDev* fits, const Tile* tiles,
                           const FitDev* one, int n_tiles, size_t lds, int32_t mode, hipStream_t s);
hipError_t launch_step_f32d(int block, int kin, const FitDev* fits, const Tile* tiles,
                            const FitDev* one, int n_tiles, size_t lds, int32_t mode, hipStream_t s);
hipError_t launch_step_f32f(int block, int kin, const FitDev* fits, const Tile* tiles,
                            const FitDev* one, int n_tiles, size_t lds, int32_t mode, hipStream_t s);
// one fit, fd (a host copy of its description) passed by value: the step
// over n_tiles tiles as tile_of splits it; the finalize jobs of that fit
// (bin jobs, then cell jobs) over n_rows tile rows
hipError_t launch_step1(bool f64, bool acc64, int block, int kin, const FitDev& fd, int n_tiles,
                        size_t lds, int32_t mode, hipStream_t s);
hipError_t launch_finalize1(bool f64, const FitDev& fd, int n_rows, int32_t mode, hipStream_t s);

// ---- prior smoothing basis (m2m_smooth.cpp) -------------------------------
// Doubles of the eigendecomposition of the thin-plate penalty of an
// n_E x n_x grid: n_E n_x eigenvalues, then the eigenvectors of its four
// reflection-parity blocks.
size_t smooth_basis_len(int nE, int nx);
// Compute it (or take it from the process-wide cache of grid shapes) into
// out; false if the eigen-iteration does not converge.
bool smooth_basis(int nE, int nx, double hE, double hx, double* out);
hipError_t launch_assign(bool f64, const FitDev* fits, const Tile* tiles, int n_tiles,
                         hipStream_t s);
hipError_t launch_weights(bool f64, const void* u, void* w, int64_t n, double scale,
                          hipStream_t s);
hipError_t launch_poke(FitState* st, int32_t steps_left, int32_t correct, hipStream_t s);
hipError_t launch_gather(const FitDev* fits, int n, int32_t* out, hipStream_t s);
hipError_t launch_residuals(bool f64, const FitDev* fit, hipStream_t s);
size_t step_lds_bytes(bool f64, bool acc64, int J, int n_r, int n_R, int n_v, int kpriv, int C,
                      int scf_nr, int scf_lmax);
int kin_class(int kin, int gh_nmax, int dens, bool scf);
int private_copies(bool f64, int J);

}  // namespace m2m

// Host side of the C ABI declared in include/m2m.h: validation, workspace
// layout, tables (bin edges, L_c(E)), graph capture of the step loop, and
// the batch of fits that step together.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "m2m.h"
#include "m2m_internal.h"

using namespace m2m;

namespace {

constexpr int kGraphSteps = 32;     // M2M steps per captured graph of one fit
constexpr int kBatchGraphSteps = 8; // of a batch (captured again when fits come and go)
constexpr int kProfileMax = 4096;   // most steps one m2m_profile_step call times
constexpr int kBatchProfileMax = 256;  // most steps one m2m_batch_profile call times
// A fit of a batch whose tile rows of observable sums take at most this many
// bytes is finalized by one block (every column and the end of its step, no
// hand-over between blocks); larger ones by column jobs.
constexpr size_t kWholeFitMaxBytes = size_t(1) << 20;
constexpr uint32_t kStateMagic = 0x4d324d31u;  // "M2M1"
constexpr uint32_t kStateVersion = 2u;         // 2: with the FP64 prior grid
constexpr double kPi = 3.14159265358979323846;

// launch shape for contexts and batches created from now on
int g_block = 1024, g_tiles_per_cu = 1;
constexpr int kGroups = 2;  // most groups a batch of two or more fits steps as
int g_groups = 2;           // groups of a batch of two or more fits (1 or 2)
int g_batch_graphs = 0;     // batches replay captured graphs (1) or launch directly (0)
int g_deposit = M2M_DEPOSIT_F64;
int g_kpriv_cap = 0;  // most private bin copies per block (0: as many as fit, at most 8)
int g_interleave = -1;  // tiles of one fit: contiguous (0), interleaved (1), by state size (-1)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

bool is_fin(double v) { return std::isfinite(v); }

int n_cus() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
        return 256;
    return n;
}

size_t max_lds() {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || n <= 0)
        return 65536;
    return (size_t)n;
}

int kin_per_annulus(const m2m_obs_layout& L) {
    switch (L.kin) {
        case M2M_KIN_NONE: return 0;
        case M2M_KIN_V2: return 1;
        case M2M_KIN_GH: return L.gh_nmax;
        case M2M_KIN_LOSVD: return L.n_v;
        default: return -1;
    }
}

// "" if the layout is valid, else the reason
std::string check_layout(const m2m_obs_layout* L) {
    if (!L) return "layout is NULL";
    if (L->n_r < 1 || L->n_r > 4096) return "n_r must be in 1..4096";
    if (!(is_fin(L->r_min) && is_fin(L->r_max) && L->r_min > 0 && L->r_max > L->r_min))
        return "need 0 < r_min < r_max";
    if (L->kin < M2M_KIN_NONE || L->kin > M2M_KIN_LOSVD) return "unknown kin";
    if (L->kin != M2M_KIN_NONE) {
        if (L->n_R < 1 || L->n_R > 4096) return "n_R must be in 1..4096";
        if (!(is_fin(L->R_min) && is_fin(L->R_max) && L->R_min > 0 && L->R_max > L->R_min))
            return "need 0 < R_min < R_max";
    } else if (L->n_R < 0 || L->n_R > 4096) {
        return "n_R must be in 0..4096";
    }
    if (L->gh_nmax < 0 || L->n_v < 0) return "gh_nmax and n_v must be >= 0";
    if (L->kin == M2M_KIN_GH && (L->gh_nmax < 1 || L->gh_nmax > kMaxGH)) return "gh_nmax must be in 1..8";
    if (L->kin == M2M_KIN_LOSVD) {
        if (L->n_v < 1 || L->n_v > kMaxLOSVD) return "n_v must be in 1..256";
        if (!(is_fin(L->v_min) && is_fin(L->v_max) && L->v_max > L->v_min)) return "need v_min < v_max";
    }
    if (L->dens != M2M_DENS_BINS && L->dens != M2M_DENS_ALM) return "unknown dens";
    if (L->dens == M2M_DENS_ALM) {
        if (L->n_r < 2) return "the a_lm mesh needs n_r >= 2 radii";
        if (L->l_max < 0 || L->l_max > kMaxLM) return "l_max must be in 0..8";
    }
    const int64_t nlm = L->dens == M2M_DENS_ALM ? (int64_t)(L->l_max + 1) * (L->l_max + 1) : 1;
    const int64_t J = (int64_t)L->n_r * nlm +
                      (int64_t)(L->kin == M2M_KIN_NONE ? 0 : L->n_R) * kin_per_annulus(*L);
    if (J > 16384) return "too many observables";
    return "";
}

// radial bins, or the intervals between the a_lm mesh radii
int radial_intervals(const m2m_obs_layout& L) {
    return L.dens == M2M_DENS_ALM ? L.n_r - 1 : L.n_r;
}

// observables of the density part: n_r bins, or (l_max + 1)^2 at each mesh radius
int32_t dens_obs(const m2m_obs_layout& L) {
    return L.dens == M2M_DENS_ALM ? L.n_r * (L.l_max + 1) * (L.l_max + 1) : L.n_r;
}

int32_t num_obs(const m2m_obs_layout& L) {
    if (L.kin == M2M_KIN_NONE) return dens_obs(L);
    return dens_obs(L) + L.n_R * kin_per_annulus(L);
}

// log10(lambda) search range of the prior smoothing and the number of
// points of its first stage (steps of 0.25)
// cell width of the prior grid along energy, in the variable the energy bins
// are linear in (E, or exp E)
double energy_width(const m2m_params& P) {
    if (P.cells & M2M_CELLS_EXP_E) return (std::exp(P.E_hi) - std::exp(P.E_lo)) / P.n_E;
    return (P.E_hi - P.E_lo) / P.n_E;
}

// cells of the prior grid: n_E n_x, twice that with the L_z split
int n_cells(const m2m_params& P) {
    return P.n_E * P.n_x * ((P.cells & M2M_CELLS_LZ) ? 2 : 1);
}

void smooth_range(const m2m_params& P, double* plo, double* phi, int* k1) {
    const double hE = energy_width(P), hx = 1.0 / P.n_x;
    double ghi = 0.0, glo = INFINITY;
    if (P.n_E > 1) {
        ghi += 4.0 / (hE * hE);
        const double s = std::sin(kPi / (2.0 * P.n_E));
        glo = std::min(glo, 4.0 * s * s / (hE * hE));
    }
    if (P.n_x > 1) {
        ghi += 4.0 / (hx * hx);
        const double s = std::sin(kPi / (2.0 * P.n_x));
        glo = std::min(glo, 4.0 * s * s / (hx * hx));
    }
    *plo = -2.0 * std::log10(ghi) - 4.0;
    *phi = -2.0 * std::log10(glo) + 4.0;
    *k1 = (int)std::floor((*phi - *plo) / 0.25) + 1;
}

std::string check_params(const m2m_params* P) {
    if (!P) return "params is NULL";
    if (!(is_fin(P->dt) && P->dt > 0)) return "dt must be > 0";
    if (!(is_fin(P->eps) && P->eps >= 0)) return "eps must be >= 0";
    if (!(is_fin(P->mu) && P->mu >= 0)) return "mu must be >= 0";
    if (!(is_fin(P->alpha) && P->alpha >= 0)) return "alpha must be >= 0";
    if (!(is_fin(P->mass) && P->mass > 0)) return "mass must be > 0";
    if (P->entropy != M2M_S_MPR && P->entropy != M2M_S_GWR) return "unknown entropy";
    if (P->n_E < 1 || P->n_x < 1 || (int64_t)P->n_E * P->n_x > kMaxCells) return "need n_E, n_x >= 1 and n_E*n_x <= 4096";
    if (P->prior_every < 0) return "prior_every must be >= 0";
    if (!(is_fin(P->E_lo) && is_fin(P->E_hi) && P->E_hi > P->E_lo)) return "need E_lo < E_hi";
    if (P->smooth != 0 && P->smooth != 1) return "smooth must be 0 or 1";
    if (P->cells & ~(M2M_CELLS_LZ | M2M_CELLS_EXP_E)) return "unknown cells flags";
    if (n_cells(*P) > kMaxCells) return "need n_E*n_x <= 2048 with the L_z split";
    if (P->smooth && (P->n_E > kSmoothMaxSide || P->n_x > kSmoothMaxSide))
        return "prior smoothing needs n_E, n_x <= 128";
    if (P->smooth && P->n_E * P->n_x > kSmoothMaxCells)
        return "prior smoothing needs n_E*n_x <= 2048";
    if (P->scf_nr != 0) {
        if (P->scf_nr < 2 || P->scf_nr > kMaxScfNodes) return "scf_nr must be 0 or 2..64";
        if (P->scf_lmax < 0 || P->scf_lmax > kMaxLM) return "scf_lmax must be 0..8";
        if (!(is_fin(P->scf_rmin) && is_fin(P->scf_rmax) && P->scf_rmin > 0 &&
              P->scf_rmax > P->scf_rmin))
            return "need 0 < scf_rmin < scf_rmax";
        if (P->scf_every < 1) return "scf_every must be >= 1";
    }
    if (P->smooth && P->n_E * P->n_x > 1) {
        double plo, phi;
        int k1;
        smooth_range(*P, &plo, &phi, &k1);
        if (k1 > kSmoothMaxPoints) return "prior smoothing: grid spacings too different";
    }
    return "";
}

std::string check_potential(const m2m_potential* p) {
    if (!p) return "potential is NULL";
    if (!(is_fin(p->G) && p->G > 0)) return "G must be > 0";
    if (!(is_fin(p->M_star) && is_fin(p->upsilon) && p->M_star * p->upsilon >= 0)) return "bad Hernquist mass";
    if (!(is_fin(p->a) && p->a > 0)) return "a must be > 0";
    if (!(is_fin(p->M200) && p->M200 >= 0)) return "M200 must be >= 0";
    if (p->M200 > 0 && !(is_fin(p->c) && p->c > 0 && is_fin(p->r_s) && p->r_s > 0))
        return "NFW needs c > 0 and r_s > 0";
    if (!(is_fin(p->v0) && p->v0 >= 0)) return "v0 must be >= 0";
    if (p->v0 > 0 && !(is_fin(p->r0) && p->r0 > 0 && is_fin(p->q) && p->q > 0))
        return "the logarithmic halo needs r0 > 0 and q > 0";
    return "";
}

// ---------------------------------------------------------------- physics --
// (independent host evaluation, FP64: bin edges and the L_c(E) table)
struct HostPot {
    double GMh, a, GM200, c, rs, fc;
    double v02, r02;  // logarithmic halo v0^2, r0^2 (v02 = 0: none)
    explicit HostPot(const m2m_potential& p) {
        GMh = p.G * p.M_star * p.upsilon;
        a = p.a;
        GM200 = p.M200 > 0 ? p.G * p.M200 : 0.0;
        c = p.c;
        rs = p.r_s;
        fc = p.M200 > 0 ? std::log1p(c) - c / (1.0 + c) : 1.0;
        v02 = p.v0 > 0 ? p.v0 * p.v0 : 0.0;
        r02 = p.v0 > 0 ? p.r0 * p.r0 : 1.0;
    }
    // on the equatorial plane at radius r (the whole potential if spherical)
    double phi(double r) const {
        double v = -GMh / (r + a);
        if (GM200 > 0) v += (r > 0) ? -GM200 / fc * std::log1p(r / rs) / r : -GM200 / (fc * rs);
        if (v02 > 0) v += 0.5 * v02 * std::log(r02 + r * r);
        return v;
    }
    double GM(double r) const {  // G M(<r)
        double m = GMh * r * r / ((r + a) * (r + a));
        if (GM200 > 0) {
            const double q = r / rs;
            m += GM200 / fc * (std::log1p(q) - q / (1.0 + q));
        }
        return m;
    }
    // squared circular speed in the equatorial plane, r dPhi/dr
    double vc2(double r) const {
        double v = r > 0 ? GM(r) / r : 0.0;
        if (v02 > 0) v += v02 * r * r / (r02 + r * r);
        return v;
    }
    double ecirc(double r) const { return phi(r) + 0.5 * vc2(r); }
    // r dE_c/dr with E_c = Phi + v_c^2 / 2: for the spherical parts
    // G M / (2 r) + (G M)' / 2, (G M)' = 2 G M a r / (r + a)^3 (Hernquist) +
    // G M200 / f(c) r / (r_s^2 (1 + r/r_s)^2); for the logarithmic halo
    // v0^2 r^2 (2 r0^2 + r^2) / (r0^2 + r^2)^2
    double decirc_dlnr(double r) const {
        const double ra = r + a;
        double d = 0.5 * GM(r) / r + GMh * a * r / (ra * ra * ra);
        if (GM200 > 0) {
            const double q1 = 1.0 + r / rs;
            d += 0.5 * GM200 / fc * r / (rs * rs * q1 * q1);
        }
        if (v02 > 0) {
            const double s = r02 + r * r;
            d += v02 * r * r * (2.0 * r02 + r * r) / (s * s);
        }
        return d;
    }
    // ln of the radius of the circular orbit with energy E (phi(0) < E < 0):
    // Newton steps in ln r from the guess x0 inside a bracket that every
    // evaluation narrows (E_c increases with r); a step that leaves the
    // bracket is replaced by bisection
    double ln_rc(double E, double x0) const {
        double lo = -60.0, hi = 60.0;
        double x = std::min(std::max(x0, lo), hi);
        for (int it = 0; it < 200; ++it) {
            const double r = std::exp(x);
            const double f = ecirc(r) - E;
            if (f < 0) lo = x; else hi = x;
            if (f == 0 || hi - lo < 1e-15) break;
            double xn = x - f / decirc_dlnr(r);
            if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
            if (std::fabs(xn - x) < 4e-16 * std::max(1.0, std::fabs(x))) {
                x = xn;
                break;
            }
            x = xn;
        }
        return x;
    }
};

double log_edge(double lo, double hi, int n, int k) {
    if (k == 0) return lo;
    if (k == n) return hi;
    return lo * std::pow(hi / lo, (double)k / (double)n);
}

double lin_edge(double lo, double hi, int n, int k) {
    if (k == 0) return lo;
    if (k == n) return hi;
    return lo + (hi - lo) * (double)k / (double)n;
}

// ln zeta range of the L_c table: zeta = (E - Phi0) / (-E)
constexpr double kLz0 = -16.1180956509583;  // ln 1e-7
constexpr double kLz1 = 20.7232658369464;   // ln 1e9
constexpr double kLzHalo1 = 3.68887945411394;  // ln 40: with the logarithmic halo, zeta <= 40

// ---------------------------------------------------------------- layout ---
struct WsLayout {
    size_t st, fd, tiles, jobs, redge2, rmesh, Redge2, vedge, Vp, isp, rp, ucell, lctab, cidx;
    size_t cdata, gprior, scf_rho, scf_sum, scf_tab, sm_basis;
    size_t Y, sigma, yv, ytil, delta, obs, hist, chi2p, partials, total;
    int seg_cap, row_len, nbj, ncj, npj, J, C, P;  // P: interval sums of the expansion
};

// entries of the node table of the self-consistent potential
size_t scf_table_len(const m2m_params& P) {
    return P.scf_nr > 0 ? (size_t)P.scf_nr * (size_t)((P.scf_lmax + 1) * (P.scf_lmax + 1)) * 2 : 0;
}

int seg_cap_of(int64_t n, int row_len) {
    // at least ~1024 particles per tile, and partial rows of at most
    // 16 bytes per particle (half the FP32 particle state)
    const int64_t by_n = (n + 1023) / 1024;
    const int64_t by_mem = (16 * n) / ((int64_t)row_len * 8);
    int64_t cap = std::min(by_n, std::max<int64_t>(by_mem, 1));
    cap = std::max<int64_t>(1, std::min<int64_t>(cap, 4096));
    cap = std::min<int64_t>(cap, std::max<int64_t>(1, n / kSegAlign));
    return (int)cap;
}

// cell_index = false: no per-particle cell index (observation only)
WsLayout plan(const m2m_obs_layout& L, const m2m_params& P, int64_t n, bool f64,
              bool cell_index = true) {
    WsLayout w{};
    const size_t sz = f64 ? 8 : 4;
    w.J = num_obs(L);
    w.C = n_cells(P);
    w.P = (int)scf_table_len(P);  // 2 K nlm interval sums, as many as table entries
    w.row_len = w.J + 2 * w.C + w.P;
    w.nbj = (w.J + kFinCols - 1) / kFinCols;
    w.ncj = (w.C + kFinCols - 1) / kFinCols;
    w.npj = (w.P + kFinCols - 1) / kFinCols;
    w.seg_cap = seg_cap_of(n, w.row_len);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    w.st = take(sizeof(FitState));
    w.fd = take(sizeof(FitDev));
    w.tiles = take(sizeof(Tile) * (size_t)w.seg_cap);
    w.jobs = take(sizeof(FinJob) * (size_t)(w.nbj + w.ncj + w.npj));
    const int nR = L.kin == M2M_KIN_NONE ? 0 : L.n_R;
    const int nv = L.kin == M2M_KIN_LOSVD ? L.n_v : 0;
    w.redge2 = take(sz * (size_t)(L.n_r + 1));
    w.rmesh = take(sz * (size_t)(L.n_r + 1));
    w.Redge2 = take(sz * (size_t)(nR + 1));
    w.vedge = take(sz * (size_t)(nv + 1));
    w.Vp = take(sz * (size_t)std::max(nR, 1));
    w.isp = take(sz * (size_t)std::max(nR, 1));
    w.rp = take(sz * (size_t)w.J);
    w.ucell = take(sz * (size_t)w.C);
    w.lctab = take(sz * (size_t)kLcTable);
    w.Y = take(8 * (size_t)w.J);
    w.sigma = take(8 * (size_t)w.J);
    w.yv = take(8 * (size_t)w.J);
    w.ytil = take(8 * (size_t)w.J);
    w.delta = take(8 * (size_t)w.J);
    w.obs = take(8 * (size_t)w.J);
    w.hist = take(8 * (size_t)kHistCap);
    w.chi2p = take(8 * (size_t)w.nbj);
    w.partials = take(8 * (size_t)w.seg_cap * (size_t)w.row_len);
    w.cidx = take(cell_index ? 2 * (size_t)n : 0);
    w.cdata = take(8 * (size_t)w.C);
    w.gprior = take(8 * (size_t)w.C);
    w.scf_rho = take(8 * (size_t)std::max(P.scf_nr, 1));
    w.scf_sum = take(8 * (size_t)std::max(w.P, 1));
    w.scf_tab = take(8 * (size_t)std::max(w.P, 1));
    // eigendecomposition of the smoothing penalty (both L_z halves share it)
    w.sm_basis = take(P.smooth ? 8 * smooth_basis_len(P.n_E, P.n_x) : 8);
    w.total = o;
    return w;
}

// The observation part of a fit's description: the kernels' layout fields
// and the workspace segments from b (contexts and the allocation-free
// observation share it).
void describe_obs(FitDev& f, const m2m_obs_layout& L, const WsLayout& w, unsigned char* b) {
    const int n_int = radial_intervals(L);
    f.n_r = n_int;
    f.jk0 = dens_obs(L);
    f.l_max = L.dens == M2M_DENS_ALM ? L.l_max : 0;
    f.n_R = L.kin == M2M_KIN_NONE ? 0 : L.n_R;
    f.kin = L.kin;
    f.nk = kin_per_annulus(L);
    f.J = w.J;
    f.n_v = L.kin == M2M_KIN_LOSVD ? L.n_v : 0;
    f.gh_nmax = L.kin == M2M_KIN_GH ? L.gh_nmax : 0;
    f.C = w.C;
    f.lr0 = std::log2(L.r_min * L.r_min);
    f.lrs = n_int / std::log2((L.r_max * L.r_max) / (L.r_min * L.r_min));
    if (f.n_R > 0) {
        f.lR0 = std::log2(L.R_min * L.R_min);
        f.lRs = L.n_R / std::log2((L.R_max * L.R_max) / (L.R_min * L.R_min));
    }
    if (f.n_v > 0) {
        f.vmin = L.v_min;
        f.vidv = L.n_v / (L.v_max - L.v_min);
    }
    f.redge2 = b + w.redge2;
    f.rmesh = b + w.rmesh;
    f.Redge2 = b + w.Redge2;
    f.vedge = b + w.vedge;
    f.Vp = b + w.Vp;
    f.isp = b + w.isp;
    f.rp = b + w.rp;
    f.Y = reinterpret_cast<double*>(b + w.Y);
    f.sigma = reinterpret_cast<double*>(b + w.sigma);
    f.yv = reinterpret_cast<double*>(b + w.yv);
    f.ytil = reinterpret_cast<double*>(b + w.ytil);
    f.delta = reinterpret_cast<double*>(b + w.delta);
    f.obs_out = reinterpret_cast<double*>(b + w.obs);
    f.partials = reinterpret_cast<double*>(b + w.partials);
    f.row_len = w.row_len;
    f.n_bin_jobs = w.nbj;
    f.n_cell_jobs = w.ncj;
    f.n_pot_jobs = w.npj;
    f.chi2_hist = reinterpret_cast<double*>(b + w.hist);
    f.chi2_part = reinterpret_cast<double*>(b + w.chi2p);
    f.st = reinterpret_cast<FitState*>(b + w.st);
}

// The observation tables (bin edges, GH centres and inverse widths) in the
// state type, written into img, the image of the workspace bytes
// [w.redge2, w.rp). V, S: n_R GH centres and widths, or NULL for 0 and 1.
template <typename T>
void put_obs_tables_t(unsigned char* img, const WsLayout& w, const m2m_obs_layout& L,
                      const double* V, const double* S) {
    auto at = [&](size_t off) { return reinterpret_cast<T*>(img + (off - w.redge2)); };
    std::memset(img, 0, w.rp - w.redge2);
    const int n_int = radial_intervals(L);
    const int nR = L.kin == M2M_KIN_NONE ? 0 : L.n_R;
    const int nv = L.kin == M2M_KIN_LOSVD ? L.n_v : 0;
    T* re2 = at(w.redge2);
    T* rm = at(w.rmesh);
    for (int k = 0; k <= n_int; ++k) {
        const double e = log_edge(L.r_min, L.r_max, n_int, k);
        rm[k] = (T)e;
        re2[k] = (T)(e * e);
    }
    T* Re2 = at(w.Redge2);
    for (int k = 0; k <= nR; ++k) {
        const double e = log_edge(L.R_min, L.R_max, L.n_R, k);
        Re2[k] = (T)(e * e);
    }
    T* ve = at(w.vedge);
    for (int k = 0; k <= nv; ++k) ve[k] = (T)lin_edge(L.v_min, L.v_max, L.n_v, k);
    T* vp = at(w.Vp);
    T* isp = at(w.isp);
    for (int p = 0; p < std::max(nR, 1); ++p) {
        vp[p] = (T)(V ? V[p] : 0.0);
        isp[p] = (T)(1.0 / (S ? S[p] : 1.0));
    }
}

void put_obs_tables(unsigned char* img, const WsLayout& w, const m2m_obs_layout& L, bool f64,
                    const double* V, const double* S) {
    if (f64)
        put_obs_tables_t<double>(img, w, L, V, S);
    else
        put_obs_tables_t<float>(img, w, L, V, S);
}

}  // namespace

// ================================================================ context ==
struct m2m_ctx {
    m2m_potential pot{};
    m2m_obs_layout lay{};
    m2m_params par{};
    int64_t n = 0;
    bool f64 = false;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    unsigned char* ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    WsLayout w{};
    FitDev fd{};
    FitDev* fd_dev = nullptr;
    FitState* st = nullptr;
    Tile* tiles = nullptr;
    FinJob* jobs = nullptr;
    int n_tiles = 0;
    int n_jobs = 0;
    size_t lds = 0;
    int block = 256, kin = 0;
    bool acc64 = true;
    bool wt = false;  // write-through particle stores (kModeWriteThrough)
    bool il = false;  // interleaved tiles in the step kernel (kModeInterleave)
    hipGraphExec_t graph_prof = nullptr;  // steps with an extra measuring reduction
    bool targets = false;
    bool ytil_init = false;
    std::vector<double> Vp, sp;  // current Gauss-Hermite centres (host)
    hipGraphExec_t graph = nullptr;
    m2m_batch* batch = nullptr;
    // set when the fit leaves a batch: recorded on the batch stream after the
    // last run that may still read the fit (its tiles skip an idle fit, but
    // they read its counters); the fit's own work that changes its state
    // waits for it first
    hipEvent_t idle_ev = nullptr;
    bool idle_pending = false;
    // false while no step can have left a prior assignment pending (a new
    // context, or one just flushed): flush_assign then reads nothing back
    bool may_assign = false;
    hipEvent_t own_ev = nullptr;  // the fit's own work, which a batch waits for at admission
    std::string err;
};

namespace {

// the calling thread's last failure of m2m_observe_noalloc (no context)
thread_local char g_na_err[256];

m2m_status fail(m2m_ctx* c, m2m_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

m2m_status hip_fail(m2m_ctx* c, hipError_t e, const char* what) {
    return fail(c, M2M_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define M2M_HIP(c, call)                                   \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return hip_fail(c, e_, #call); \
    } while (0)

template <typename T>
std::vector<unsigned char> as_bytes(const std::vector<double>& v) {
    std::vector<unsigned char> out(v.size() * sizeof(T));
    for (size_t i = 0; i < v.size(); ++i) {
        const T t = (T)v[i];
        std::memcpy(out.data() + i * sizeof(T), &t, sizeof(T));
    }
    return out;
}

// A copy ordered on the context's stream, complete on return (host
// buffers may be reused at once).
hipError_t copy_sync(hipStream_t s, void* dst, const void* src, size_t n, hipMemcpyKind kind) {
    hipError_t e = hipMemcpyAsync(dst, src, n, kind, s);
    return e == hipSuccess ? hipStreamSynchronize(s) : e;
}

m2m_status upload(m2m_ctx* c, size_t off, const std::vector<double>& v) {
    std::vector<unsigned char> b = c->f64 ? as_bytes<double>(v) : as_bytes<float>(v);
    if (b.empty()) return M2M_OK;
    M2M_HIP(c, copy_sync(c->stream, c->ws + off, b.data(), b.size(), hipMemcpyHostToDevice));
    return M2M_OK;
}

m2m_status upload64(m2m_ctx* c, size_t off, const std::vector<double>& v) {
    if (v.empty()) return M2M_OK;
    M2M_HIP(c, copy_sync(c->stream, c->ws + off, v.data(), v.size() * sizeof(double),
                         hipMemcpyHostToDevice));
    return M2M_OK;
}

m2m_status upload_gh(m2m_ctx* c, const std::vector<double>& V, const std::vector<double>& S) {
    std::vector<double> isp(S.size());
    for (size_t i = 0; i < S.size(); ++i) isp[i] = 1.0 / S[i];
    m2m_status s = upload(c, c->w.Vp, V);
    if (s != M2M_OK) return s;
    return upload(c, c->w.isp, isp);
}

// Split [0, n) into `count` tiles of near-equal size with aligned boundaries.
void split_tiles(int64_t n, int count, int fit, int row0, std::vector<Tile>& out) {
    for (int t = 0; t < count; ++t) out.push_back(tile_of(n, t, count, fit, row0));
}

void fin_jobs(const WsLayout& w, int fit, int n_rows, std::vector<FinJob>& out) {
    for (int b = 0; b < w.nbj; ++b) out.push_back(FinJob{fit, 0, b * kFinCols, n_rows});
    for (int b = 0; b < w.ncj; ++b) out.push_back(FinJob{fit, 1, b * kFinCols, n_rows});
    for (int b = 0; b < w.npj; ++b) out.push_back(FinJob{fit, 2, b * kFinCols, n_rows});
}

m2m_status sync(m2m_ctx* c) {
    M2M_HIP(c, hipStreamSynchronize(c->stream));
    return M2M_OK;
}

// Work that changes the fit's state waits (on the device) for the batch
// runs that may still read it after it left a batch.
m2m_status after_batch(m2m_ctx* c) {
    if (c->idle_pending) {
        M2M_HIP(c, hipStreamWaitEvent(c->stream, c->idle_ev, 0));
        c->idle_pending = false;
    }
    return M2M_OK;
}

m2m_status read_state(m2m_ctx* c, FitState& s) {
    M2M_HIP(c, hipStreamSynchronize(c->stream));
    M2M_HIP(c, copy_sync(c->stream, &s, c->st, sizeof(FitState), hipMemcpyDeviceToHost));
    return M2M_OK;
}

// Assign cell priors computed by the last refresh, if still pending.
m2m_status flush_assign(m2m_ctx* c) {
    if (!c->may_assign) return M2M_OK;
    FitState s{};
    m2m_status r = read_state(c, s);
    if (r != M2M_OK) return r;
    if (s.assign_pending) {
        M2M_HIP(c, launch_assign(c->f64, c->fd_dev, c->tiles, c->n_tiles, c->stream));
        if ((r = sync(c)) != M2M_OK) return r;
    }
    c->may_assign = false;
    return M2M_OK;
}

m2m_status check_error(m2m_ctx* c) {
    FitState s{};
    m2m_status r = read_state(c, s);
    if (r != M2M_OK) return r;
    if (s.error & 1) return fail(c, M2M_ENONFINITE, "chi^2 became non-finite");
    return M2M_OK;
}

// Rebuild the self-consistent potential from the current state: the step
// kernel deposits the interval sums only, the finalize reduces them and
// writes the node table.
m2m_status refresh_potential(m2m_ctx* c) {
    M2M_HIP(c, launch_step1(c->f64, c->acc64, c->block, c->kin, c->fd, c->n_tiles, c->lds,
                           kModePot, c->stream));
    M2M_HIP(c, launch_finalize1(c->f64, c->fd, c->n_tiles, kModePot, c->stream));
    return M2M_OK;
}

// One M2M step: the step kernel over all tiles, then the finalize.
hipError_t launch_one_step(m2m_ctx* c, hipStream_t s) {
    hipError_t e = launch_step1(c->f64, c->acc64, c->block, c->kin, c->fd, c->n_tiles, c->lds,
                               kModeStep | (c->wt ? kModeWriteThrough : 0) |
                                   (c->il ? kModeInterleave : 0),
                               s);
    if (e == hipSuccess) e = launch_finalize1(c->f64, c->fd, c->n_tiles, kModeStep, s);
    return e;
}

// Capture n repetitions of body(stream) on the capture stream, instantiate
// them as one graph and upload it on stream `up`, so that its first launch
// costs no more than the later ones.
template <typename F>
hipError_t capture_steps(hipStream_t cap, int n, F body, hipGraphExec_t* out, hipStream_t up) {
    *out = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    for (int k = 0; k < n && e == hipSuccess; ++k) e = body(cap);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(cap, &g);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e == hipSuccess) e = hipGraphUpload(*out, up);
    if (e != hipSuccess) {
        if (*out) (void)hipGraphExecDestroy(*out);
        *out = nullptr;
    }
    return e;
}

m2m_status ensure_graph(m2m_ctx* c) {
    if (c->graph) return M2M_OK;
    if (!c->cap) M2M_HIP(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    const hipError_t e = capture_steps(
        c->cap, kGraphSteps,
        [c](hipStream_t s) { return launch_one_step(c, s); }, &c->graph, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "step graph");
    return M2M_OK;
}


// Steps as in the step graph, each followed by one more reduction in the
// measuring mode that changes no state (m2m_profile_step).
m2m_status ensure_prof_graph(m2m_ctx* c) {
    if (c->graph_prof) return M2M_OK;
    if (!c->cap) M2M_HIP(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
    const hipError_t e = capture_steps(
        c->cap, kGraphSteps,
        [c](hipStream_t s) {
            hipError_t r = launch_one_step(c, s);
            if (r == hipSuccess)
                r = launch_finalize1(c->f64, c->fd, c->n_tiles, kModeObserve, s);
            return r;
        },
        &c->graph_prof, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "profile graph");
    return M2M_OK;
}

}  // namespace

extern "C" {

int32_t m2m_num_observables(const m2m_obs_layout* layout) {
    if (!check_layout(layout).empty()) return 0;
    return num_obs(*layout);
}

size_t m2m_workspace_bytes(const m2m_obs_layout* layout, const m2m_params* params, int64_t n,
                           int32_t dtype) {
    if (!check_layout(layout).empty() || !check_params(params).empty() || n < 1) return 0;
    if (dtype != M2M_F32 && dtype != M2M_F64) return 0;
    return plan(*layout, *params, n, dtype == M2M_F64).total;
}

m2m_status m2m_set_launch(int32_t block, int32_t tiles_per_cu) {
    if (block != 256 && block != 512 && block != 1024) return M2M_EINVAL;
    if (tiles_per_cu < 1 || tiles_per_cu > 16) return M2M_EINVAL;
    g_block = block;
    g_tiles_per_cu = tiles_per_cu;
    return M2M_OK;
}

m2m_status m2m_set_batch_graphs(int32_t on) {
    if (on != 0 && on != 1) return M2M_EINVAL;
    g_batch_graphs = on;
    return M2M_OK;
}

int32_t m2m_get_batch_graphs(void) { return g_batch_graphs; }

m2m_status m2m_set_private_copies(int32_t copies) {
    if (copies != 0 && copies != 1 && copies != 2 && copies != 4 && copies != 8) return M2M_EINVAL;
    g_kpriv_cap = copies;
    return M2M_OK;
}

int32_t m2m_get_private_copies(void) { return g_kpriv_cap; }

m2m_status m2m_set_batch_groups(int32_t groups) {
    if (groups < 1 || groups > kGroups) return M2M_EINVAL;
    g_groups = groups;
    return M2M_OK;
}

int32_t m2m_get_batch_groups(void) { return g_groups; }

m2m_status m2m_set_deposit_mode(int32_t mode) {
    if (mode != M2M_DEPOSIT_F64 && mode != M2M_DEPOSIT_F32_COMPENSATED) return M2M_EINVAL;
    g_deposit = mode;
    return M2M_OK;
}

int32_t m2m_get_deposit_mode(void) { return g_deposit; }

m2m_status m2m_set_interleave(int32_t mode) {
    if (mode < -1 || mode > 1) return M2M_EINVAL;
    g_interleave = mode;
    return M2M_OK;
}

int32_t m2m_get_interleave(void) { return g_interleave; }

m2m_status m2m_get_launch(int32_t* block, int32_t* tiles_per_cu) {
    if (block) *block = g_block;
    if (tiles_per_cu) *tiles_per_cu = g_tiles_per_cu;
    return M2M_OK;
}

const char* m2m_last_error(const m2m_ctx* ctx) {
    if (!ctx) return g_na_err[0] ? g_na_err : "context is NULL";
    return ctx->err.c_str();
}

m2m_status m2m_create(const m2m_potential* pot, const m2m_obs_layout* layout,
                      const m2m_params* params, int64_t n, int32_t dtype, void* x, void* y,
                      void* z, void* vx, void* vy, void* vz, void* u, void* u_prior,
                      void* workspace, size_t workspace_bytes, void* hip_stream, m2m_ctx** out) {
    if (!out) return M2M_EINVAL;
    *out = nullptr;
    std::string why = check_potential(pot);
    if (why.empty()) why = check_layout(layout);
    if (why.empty()) why = check_params(params);
    if (!why.empty()) return M2M_EINVAL;
    if (n < 1 || (dtype != M2M_F32 && dtype != M2M_F64)) return M2M_EINVAL;
    void* ptrs[8] = {x, y, z, vx, vy, vz, u, u_prior};
    for (void* p : ptrs)
        if (!p || (reinterpret_cast<uintptr_t>(p) & 15u)) return M2M_EINVAL;

    m2m_ctx* c = new (std::nothrow) m2m_ctx();
    if (!c) return M2M_ENOMEM;
    c->pot = *pot;
    c->lay = *layout;
    c->par = *params;
    c->n = n;
    c->f64 = dtype == M2M_F64;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->block = c->f64 ? 256 : g_block;
    c->kin = kin_class(c->lay.kin, c->lay.gh_nmax, c->lay.dens, c->par.scf_nr > 0);
    c->w = plan(c->lay, c->par, n, c->f64);
    const WsLayout& w = c->w;
    const int kpriv = g_kpriv_cap > 0 ? std::min(private_copies(c->f64, w.J), g_kpriv_cap)
                                      : private_copies(c->f64, w.J);
    c->acc64 = c->f64 || g_deposit == M2M_DEPOSIT_F64;
    c->wt = (size_t)n * 8 * (c->f64 ? 8 : 4) <= kWriteThroughMax;
    // interleaved particle indices are 32-bit: n + n_tiles * block stays below 2^31
    c->il = (g_interleave < 0 ? (size_t)n * 8 * (c->f64 ? 8 : 4) > kStreamMin : g_interleave == 1) &&
            n < (int64_t(1) << 30);
    c->lds = step_lds_bytes(c->f64, c->acc64, w.J, radial_intervals(c->lay),
                            c->lay.kin == M2M_KIN_NONE ? 0 : c->lay.n_R,
                            c->lay.kin == M2M_KIN_LOSVD ? c->lay.n_v : 0, kpriv, w.C,
                            c->par.scf_nr, c->par.scf_lmax);
    if (c->lds > max_lds()) {
        delete c;
        return M2M_EUNSUPPORTED;
    }
    if (workspace) {
        if (workspace_bytes < w.total || (reinterpret_cast<uintptr_t>(workspace) & 255u)) {
            delete c;
            return M2M_EINVAL;
        }
        c->ws = static_cast<unsigned char*>(workspace);
        c->ws_bytes = workspace_bytes;
    } else {
        void* p = nullptr;
        if (hipMalloc(&p, w.total) != hipSuccess) {
            delete c;
            return M2M_ENOMEM;
        }
        c->ws = static_cast<unsigned char*>(p);
        c->ws_bytes = w.total;
        c->own_ws = true;
    }
    auto bail = [&](m2m_status s) {
        if (c->own_ws) (void)hipFree(c->ws);
        delete c;
        return s;
    };
    if (hipMemsetAsync(c->ws, 0, w.total, c->stream) != hipSuccess) return bail(M2M_EDEVICE);

    // ---- static description
    FitDev& f = c->fd;
    f.x = x; f.y = y; f.z = z; f.vx = vx; f.vy = vy; f.vz = vz; f.u = u; f.uh = u_prior;
    f.n = n;
    const HostPot hp(c->pot);
    f.GMh = hp.GMh;
    f.a = hp.a;
    f.GMn = hp.GM200 > 0 ? hp.GM200 / hp.fc : 0.0;
    f.rs = hp.GM200 > 0 ? hp.rs : 1.0;
    f.phi0 = hp.phi(0.0);
    const m2m_obs_layout& L = c->lay;
    unsigned char* b = c->ws;
    describe_obs(f, L, w, b);
    f.kpriv = kpriv;
    f.scf_nr = c->par.scf_nr;
    f.scf_lmax = c->par.scf_nr > 0 ? c->par.scf_lmax : 0;
    f.scf_every = std::max(c->par.scf_every, 1);
    f.scf_col0 = w.J + 2 * w.C;
    f.scf_P = w.P;
    if (c->par.scf_nr > 0) {
        f.scf_ls0 = std::log(c->par.scf_rmin);
        f.scf_ih = (c->par.scf_nr - 1) / std::log(c->par.scf_rmax / c->par.scf_rmin);
    }
    f.scf_c = c->pot.G * c->pot.upsilon * c->par.mass / (double)n;
    f.scf_rho = reinterpret_cast<double*>(b + w.scf_rho);
    f.scf_sum = reinterpret_cast<double*>(b + w.scf_sum);
    f.scf_tab = reinterpret_cast<double*>(b + w.scf_tab);
    f.entropy = c->par.entropy;
    f.n_E = c->par.n_E;
    f.n_x = c->par.n_x;
    f.prior_every = c->par.prior_every;
    f.E_lo = c->par.E_lo;
    f.E_hi = c->par.E_hi;
    f.E_scale = c->par.n_E / (c->par.E_hi - c->par.E_lo);
    f.cell_flags = c->par.cells;
    f.cell_half = c->par.n_E * c->par.n_x;
    if (c->par.cells & M2M_CELLS_EXP_E) {
        f.cell_e0 = std::exp(c->par.E_lo);
        f.cell_es = c->par.n_E / (std::exp(c->par.E_hi) - std::exp(c->par.E_lo));
    } else {
        f.cell_e0 = c->par.E_lo;
        f.cell_es = f.E_scale;
    }
    f.sm_hE = energy_width(c->par);
    f.ucell = b + w.ucell;
    f.lctab = b + w.lctab;
    f.cidx = reinterpret_cast<uint16_t*>(b + w.cidx);
    f.cdata = reinterpret_cast<double*>(b + w.cdata);
    f.gprior = reinterpret_cast<double*>(b + w.gprior);
    f.smooth = c->par.smooth;
    f.sm_basis = reinterpret_cast<double*>(b + w.sm_basis);
    if (c->par.smooth) {
        int k1 = 0;
        smooth_range(c->par, &f.sm_plo, &f.sm_phi, &k1);
        f.sm_k1 = k1;
    }
    // L_c table over ln zeta: zeta = (E - Phi(0)) / (-E), or with the
    // logarithmic halo (nothing escapes) zeta = (E - Phi(0)) / v0^2
    const double lz1 = hp.v02 > 0 ? kLzHalo1 : kLz1;
    f.lz0 = kLz0;
    f.ilz = (kLcTable - 1) / (lz1 - kLz0);
    f.hv2 = hp.v02;
    f.hr02 = hp.r02;
    f.hiq2 = hp.v02 > 0 ? 1.0 / (c->pot.q * c->pot.q) : 1.0;
    const double dt = c->par.dt;
    f.dt = dt;
    f.w0 = c->par.mass / (double)n;
    f.foc_mu = c->par.eps * dt * c->par.mu;
    f.foc_cs = c->par.entropy == M2M_S_GWR ? 1.0 : 0.0;
    f.foc_chi = c->par.eps * dt * f.w0;
    f.q = -std::expm1(-c->par.alpha * dt);
    c->fd_dev = reinterpret_cast<FitDev*>(b + w.fd);
    c->st = f.st;
    c->tiles = reinterpret_cast<Tile*>(b + w.tiles);
    c->jobs = reinterpret_cast<FinJob*>(b + w.jobs);

    // ---- tables
    std::vector<double> lct(kLcTable);
    const double phi0 = hp.phi(0.0);
    double guess = std::log(hp.a) + kLz0 * 0.5;  // small zeta: r_c ~ a sqrt(zeta)
    for (int k = 0; k < kLcTable; ++k) {
        const double lz = kLz0 + (lz1 - kLz0) * k / (kLcTable - 1);
        const double E = hp.v02 > 0 ? phi0 + hp.v02 * std::exp(lz) : phi0 / (1.0 + std::exp(lz));
        lct[k] = hp.ln_rc(E, guess);
        guess = lct[k];
    }
    std::vector<double> ones(w.C, 1.0);
    c->Vp.assign(std::max(f.n_R, 1), 0.0);
    c->sp.assign(std::max(f.n_R, 1), 1.0);
    m2m_status s = M2M_OK;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return bail(M2M_EDEVICE);
    {
        // bin edges, the a_lm mesh radii and the GH tables, one image
        std::vector<unsigned char> img(w.rp - w.redge2);
        put_obs_tables(img.data(), w, L, c->f64, nullptr, nullptr);
        if (copy_sync(c->stream, c->ws + w.redge2, img.data(), img.size(), hipMemcpyHostToDevice) !=
            hipSuccess)
            return bail(M2M_EDEVICE);
    }
    if ((s = upload(c, w.lctab, lct)) != M2M_OK) return bail(s);
    if (c->par.scf_nr > 0) {
        // nodes of the self-consistent potential, FP64
        std::vector<double> rho(c->par.scf_nr);
        for (int k = 0; k < c->par.scf_nr; ++k)
            rho[k] = log_edge(c->par.scf_rmin, c->par.scf_rmax, c->par.scf_nr - 1, k);
        if ((s = upload64(c, w.scf_rho, rho)) != M2M_OK) return bail(s);
    }
    if (c->par.smooth) {
        // the smoothing penalty's eigendecomposition for this grid shape
        std::vector<double> basis(smooth_basis_len(c->par.n_E, c->par.n_x));
        if (!smooth_basis(c->par.n_E, c->par.n_x, f.sm_hE, 1.0 / c->par.n_x, basis.data()))
            return bail(M2M_EDEVICE);
        if ((s = upload64(c, w.sm_basis, basis)) != M2M_OK) return bail(s);
    }
    if ((s = upload(c, w.ucell, ones)) != M2M_OK) return bail(s);
    if ((s = upload64(c, w.gprior, ones)) != M2M_OK) return bail(s);
    if ((s = upload_gh(c, c->Vp, c->sp)) != M2M_OK) return bail(s);

    // ---- tiles of this fit alone
    const int target = std::max(1, g_tiles_per_cu * n_cus());
    const int count = std::max(1, std::min(w.seg_cap, target));
    std::vector<Tile> tl;
    split_tiles(n, count, 0, 0, tl);
    std::vector<FinJob> jb;
    fin_jobs(w, 0, count, jb);
    c->n_tiles = (int)tl.size();
    c->n_jobs = (int)jb.size();
    if (copy_sync(c->stream, c->tiles, tl.data(), sizeof(Tile) * tl.size(), hipMemcpyHostToDevice) != hipSuccess ||
        copy_sync(c->stream, c->jobs, jb.data(), sizeof(FinJob) * jb.size(), hipMemcpyHostToDevice) != hipSuccess ||
        copy_sync(c->stream, c->fd_dev, &f, sizeof(FitDev), hipMemcpyHostToDevice) != hipSuccess)
        return bail(M2M_EDEVICE);
    *out = c;
    return M2M_OK;
}

m2m_status m2m_set_targets(m2m_ctx* c, int32_t J, const double* Y, const double* sigma,
                           const double* V_p, const double* sigma_p) {
    if (!c) return M2M_EINVAL;
    if (c->batch) return fail(c, M2M_ESTATE, "fit is in a batch");
    if (m2m_status w_ = after_batch(c); w_ != M2M_OK) return w_;
    if (J != c->w.J) return fail(c, M2M_EINVAL, "J does not match the layout");
    if (!Y || !sigma) return fail(c, M2M_EINVAL, "Y and sigma are required");
    for (int j = 0; j < J; ++j)
        if (!is_fin(Y[j]) || !is_fin(sigma[j]) || !(sigma[j] > 0))
            return fail(c, M2M_EINVAL, "targets must be finite with sigma > 0");
    std::vector<double> V = c->Vp, S = c->sp;
    if (c->lay.kin == M2M_KIN_GH) {
        if (!V_p || !sigma_p) return fail(c, M2M_EINVAL, "Gauss-Hermite layout needs V_p and sigma_p");
        for (int p = 0; p < c->fd.n_R; ++p) {
            if (!is_fin(V_p[p]) || !is_fin(sigma_p[p]) || !(sigma_p[p] > 0))
                return fail(c, M2M_EINVAL, "V_p, sigma_p must be finite with sigma_p > 0");
            V[p] = V_p[p];
            S[p] = sigma_p[p];
        }
    }
    m2m_status s = sync(c);
    if (s != M2M_OK) return s;
    M2M_HIP(c, copy_sync(c->stream, c->fd.Y, Y, sizeof(double) * J, hipMemcpyHostToDevice));
    M2M_HIP(c, copy_sync(c->stream, c->fd.sigma, sigma, sizeof(double) * J, hipMemcpyHostToDevice));
    c->Vp = V;
    c->sp = S;
    if ((s = upload_gh(c, V, S)) != M2M_OK) return s;
    if (!c->ytil_init) {
        if (c->par.scf_nr > 0 && (s = refresh_potential(c)) != M2M_OK) return s;
        M2M_HIP(c, launch_step1(c->f64, c->acc64, c->block, c->kin, c->fd, c->n_tiles, c->lds,
                               kModeInit, c->stream));
        M2M_HIP(c, launch_finalize1(c->f64, c->fd, c->n_tiles, kModeInit, c->stream));
        c->ytil_init = true;
    } else {
        M2M_HIP(c, launch_residuals(c->f64, c->fd_dev, c->stream));
    }
    c->targets = true;
    return check_error(c);
}

m2m_status m2m_step(m2m_ctx* c, int32_t n_steps, int32_t correct) {
    if (!c) return M2M_EINVAL;
    if (c->batch) return fail(c, M2M_ESTATE, "fit is in a batch");
    if (m2m_status w_ = after_batch(c); w_ != M2M_OK) return w_;
    if (!c->targets) return fail(c, M2M_ESTATE, "set targets first");
    if (n_steps < 0) return fail(c, M2M_EINVAL, "n_steps must be >= 0");
    if (n_steps == 0) return M2M_OK;
    c->may_assign = true;
    M2M_HIP(c, launch_poke(c->st, n_steps, correct ? 1 : 0, c->stream));
    const int full = n_steps / kGraphSteps, rem = n_steps % kGraphSteps;
    if (full > 0) {
        m2m_status s = ensure_graph(c);
        if (s != M2M_OK) return s;
        for (int k = 0; k < full; ++k) M2M_HIP(c, hipGraphLaunch(c->graph, c->stream));
    }
    // the rest as direct launches: a graph launch has a fixed cost of
    // several kernel launches
    for (int k = 0; k < rem; ++k) M2M_HIP(c, launch_one_step(c, c->stream));
    return M2M_OK;
}

m2m_status m2m_refresh_potential(m2m_ctx* c) {
    if (!c) return M2M_EINVAL;
    if (c->batch) return fail(c, M2M_ESTATE, "fit is in a batch");
    if (m2m_status w_ = after_batch(c); w_ != M2M_OK) return w_;
    if (c->par.scf_nr <= 0) return fail(c, M2M_EINVAL, "the fit has no self-consistent potential");
    return refresh_potential(c);
}

m2m_status m2m_get_potential(m2m_ctx* c, double* out, int32_t max) {
    if (!c || !out) return M2M_EINVAL;
    if (c->batch) return fail(c, M2M_ESTATE, "fit is in a batch");
    const size_t ST = scf_table_len(c->par);
    if (ST == 0) return fail(c, M2M_EINVAL, "the fit has no self-consistent potential");
    if (max < 0 || (size_t)max < ST) return fail(c, M2M_EINVAL, "output too small");
    m2m_status s = sync(c);
    if (s != M2M_OK) return s;
    M2M_HIP(c, copy_sync(c->stream, out, c->fd.scf_tab, 8 * ST, hipMemcpyDeviceToHost));
    return M2M_OK;
}

m2m_status m2m_update_priors(m2m_ctx* c) {
    if (!c) return M2M_EINVAL;
    if (c->batch) return fail(c, M2M_ESTATE, "fit is in a batch");
    if (m2m_status w_ = after_batch(c); w_ != M2M_OK) return w_;
    if (c->par.entropy != M2M_S_MPR) return fail(c, M2M_EINVAL, "moving priors need M2M_S_MPR");
    c->may_assign = true;
    M2M_HIP(c, launch_step1(c->f64, c->acc64, c->block, c->kin, c->fd, c->n_tiles, c->lds,
                           kModeCells, c->stream));
    M2M_HIP(c, launch_finalize1(c->f64, c->fd, c->n_tiles, kModeCells, c->stream));
    M2M_HIP(c, launch_assign(c->f64, c->fd_dev, c->tiles, c->n_tiles, c->stream));
    return M2M_OK;
}

m2m_status m2m_get_weights(m2m_ctx* c, void* dst, int32_t dst_is_device) {
    if (!c || !dst) return M2M_EINVAL;
    if (c->batch) return fail(c, M2M_ESTATE, "fit is in a batch");
    m2m_status s = flush_assign(c);
    if (s != M2M_OK) return s;
    const double scale = c->par.mass / (double)c->n;
    if (dst_is_device) {
        M2M_HIP(c, launch_weights(c->f64, c->fd.u, dst, c->n, scale, c->stream));
        s = sync(c);
    } else {
        const size_t sz = c->f64 ? 8 : 4;
        M2M_HIP(c, copy_sync(c->stream, dst, c->fd.u, sz * (size_t)c->n, hipMemcpyDeviceToHost));
        if (c->f64) {
            double* d = static_cast<double*>(dst);
            for (int64_t i = 0; i < c->n; ++i) d[i] *= scale;
        } else {
            float* d = static_cast<float*>(dst);
            for (int64_t i = 0; i < c->n; ++i) d[i] = (float)((double)d[i] * scale);
        }
    }
    if (s != M2M_OK) return s;
    return check_error(c);
}

m2m_status m2m_get_observables(m2m_ctx* c, double* y, double* y_tilde, double* delta,
                               double* chi2) {
    if (!c) return M2M_EINVAL;
    if (c->batch) return fail(c, M2M_ESTATE, "fit is in a batch");
    FitState st{};
    m2m_status s = read_state(c, st);
    if (s != M2M_OK) return s;
    const size_t J = (size_t)c->w.J;
    if (y) M2M_HIP(c, copy_sync(c->stream, y, c->fd.yv, 8 * J, hipMemcpyDeviceToHost));
    if (y_tilde) M2M_HIP(c, copy_sync(c->stream, y_tilde, c->fd.ytil, 8 * J, hipMemcpyDeviceToHost));
    if (delta) M2M_HIP(c, copy_sync(c->stream, delta, c->fd.delta, 8 * J, hipMemcpyDeviceToHost));
    if (chi2) *chi2 = st.chi2;
    if (st.error & 1) return fail(c, M2M_ENONFINITE, "chi^2 became non-finite");
    return M2M_OK;
}

m2m_status m2m_get_chi2_history(m2m_ctx* c, double* out, int32_t max, int32_t* n_out) {
    if (!c || !n_out || max < 0 || (max > 0 && !out)) return M2M_EINVAL;
    if (c->batch) return fail(c, M2M_ESTATE, "fit is in a batch");
    FitState st{};
    m2m_status s = read_state(c, st);
    if (s != M2M_OK) return s;
    std::vector<double> ring(kHistCap);
    M2M_HIP(c, copy_sync(c->stream, ring.data(), c->fd.chi2_hist, 8 * (size_t)kHistCap, hipMemcpyDeviceToHost));
    const int64_t have = std::min<int64_t>(st.tstep, kHistCap);
    const int64_t take = std::min<int64_t>(have, max);
    for (int64_t k = 0; k < take; ++k) {
        const int64_t t = st.tstep - take + k;
        out[k] = ring[(size_t)(t % kHistCap)];
    }
    *n_out = (int32_t)take;
    return M2M_OK;
}

m2m_status m2m_observe(m2m_ctx* c, const double* V_p, const double* sigma_p, double* y) {
    if (!c || !y) return M2M_EINVAL;
    if (c->batch) return fail(c, M2M_ESTATE, "fit is in a batch");
    if (m2m_status w_ = after_batch(c); w_ != M2M_OK) return w_;
    const bool tmp = c->lay.kin == M2M_KIN_GH && V_p && sigma_p;
    m2m_status s = sync(c);
    if (s != M2M_OK) return s;
    if (tmp) {
        std::vector<double> V(V_p, V_p + c->fd.n_R), S(sigma_p, sigma_p + c->fd.n_R);
        for (int p = 0; p < c->fd.n_R; ++p)
            if (!is_fin(V[p]) || !is_fin(S[p]) || !(S[p] > 0))
                return fail(c, M2M_EINVAL, "V_p, sigma_p must be finite with sigma_p > 0");
        if ((s = upload_gh(c, V, S)) != M2M_OK) return s;
    }
    M2M_HIP(c, launch_step1(c->f64, c->acc64, c->block, c->kin, c->fd, c->n_tiles, c->lds,
                           kModeObserve, c->stream));
    M2M_HIP(c, launch_finalize1(c->f64, c->fd, c->n_tiles, kModeObserve, c->stream));
    if ((s = sync(c)) != M2M_OK) return s;
    M2M_HIP(c, copy_sync(c->stream, y, c->fd.obs_out, 8 * (size_t)c->w.J, hipMemcpyDeviceToHost));
    if (tmp && (s = upload_gh(c, c->Vp, c->sp)) != M2M_OK) return s;
    return M2M_OK;
}

namespace {
struct StateHeader {
    uint32_t magic, version;
    int64_t n;
    int32_t J, C, dtype, n_R;
    int32_t targets, ytil_init, pad0, pad1;
};
}  // namespace

m2m_status m2m_get_state(m2m_ctx* c, void* host_blob, size_t* bytes) {
    if (!c || !bytes) return M2M_EINVAL;
    if (c->batch) return fail(c, M2M_ESTATE, "fit is in a batch");
    const size_t J = (size_t)c->w.J, C = (size_t)c->w.C, nR = c->Vp.size();
    const size_t sz = c->f64 ? 8 : 4;
    const size_t ST = scf_table_len(c->par);
    const size_t need = sizeof(StateHeader) + sizeof(FitState) + 8 * (5 * J + 2 * nR) +
                        sz * (C + J) + 8 * (size_t)kHistCap + 8 * C + 8 * ST;
    if (!host_blob) {
        *bytes = need;
        return M2M_OK;
    }
    if (*bytes < need) return fail(c, M2M_EINVAL, "state buffer too small");
    // a saved state never has an assignment pending: the cell of each
    // particle is kept in the workspace, not in the state
    m2m_status s = flush_assign(c);
    if (s != M2M_OK) return s;
    unsigned char* p = static_cast<unsigned char*>(host_blob);
    StateHeader h{kStateMagic, kStateVersion, c->n, (int32_t)J, (int32_t)C, c->f64 ? 1 : 0, (int32_t)nR,
                  c->targets ? 1 : 0, c->ytil_init ? 1 : 0, 0, 0};
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    M2M_HIP(c, copy_sync(c->stream, p, c->st, sizeof(FitState), hipMemcpyDeviceToHost));
    p += sizeof(FitState);
    double* const dev[5] = {c->fd.ytil, c->fd.yv, c->fd.delta, c->fd.Y, c->fd.sigma};
    for (double* d : dev) {
        M2M_HIP(c, copy_sync(c->stream, p, d, 8 * J, hipMemcpyDeviceToHost));
        p += 8 * J;
    }
    std::memcpy(p, c->Vp.data(), 8 * nR);
    p += 8 * nR;
    std::memcpy(p, c->sp.data(), 8 * nR);
    p += 8 * nR;
    M2M_HIP(c, copy_sync(c->stream, p, c->fd.ucell, sz * C, hipMemcpyDeviceToHost));
    p += sz * C;
    M2M_HIP(c, copy_sync(c->stream, p, c->fd.rp, sz * J, hipMemcpyDeviceToHost));
    p += sz * J;
    M2M_HIP(c, copy_sync(c->stream, p, c->fd.chi2_hist, 8 * (size_t)kHistCap, hipMemcpyDeviceToHost));
    p += 8 * (size_t)kHistCap;
    M2M_HIP(c, copy_sync(c->stream, p, c->fd.gprior, 8 * C, hipMemcpyDeviceToHost));
    p += 8 * C;
    if (ST > 0) M2M_HIP(c, copy_sync(c->stream, p, c->fd.scf_tab, 8 * ST, hipMemcpyDeviceToHost));
    *bytes = need;
    return M2M_OK;
}

m2m_status m2m_set_state(m2m_ctx* c, const void* host_blob, size_t bytes) {
    if (!c || !host_blob) return M2M_EINVAL;
    if (c->batch) return fail(c, M2M_ESTATE, "fit is in a batch");
    if (m2m_status w_ = after_batch(c); w_ != M2M_OK) return w_;
    size_t need = 0;
    m2m_get_state(c, nullptr, &need);
    if (bytes < need) return fail(c, M2M_EINVAL, "state blob too small");
    const unsigned char* p = static_cast<const unsigned char*>(host_blob);
    StateHeader h{};
    std::memcpy(&h, p, sizeof h);
    const size_t J = (size_t)c->w.J, C = (size_t)c->w.C, nR = c->Vp.size();
    if (h.magic != kStateMagic || h.version != kStateVersion || h.n != c->n || h.J != (int32_t)J ||
        h.C != (int32_t)C || h.dtype != (c->f64 ? 1 : 0) || h.n_R != (int32_t)nR)
        return fail(c, M2M_EINVAL, "state blob does not match this context");
    p += sizeof h;
    m2m_status s = sync(c);
    if (s != M2M_OK) return s;
    FitState st{};
    std::memcpy(&st, p, sizeof st);
    st.ticket = 0;
    st.mticket = 0;
    st.steps_left = 0;
    st.assign_pending = 0;
    M2M_HIP(c, copy_sync(c->stream, c->st, &st, sizeof st, hipMemcpyHostToDevice));
    p += sizeof(FitState);
    double* const dev[5] = {c->fd.ytil, c->fd.yv, c->fd.delta, c->fd.Y, c->fd.sigma};
    for (double* d : dev) {
        M2M_HIP(c, copy_sync(c->stream, d, p, 8 * J, hipMemcpyHostToDevice));
        p += 8 * J;
    }
    std::vector<double> V(nR), S(nR);
    std::memcpy(V.data(), p, 8 * nR);
    p += 8 * nR;
    std::memcpy(S.data(), p, 8 * nR);
    p += 8 * nR;
    c->Vp = V;
    c->sp = S;
    if ((s = upload_gh(c, V, S)) != M2M_OK) return s;
    M2M_HIP(c, copy_sync(c->stream, c->fd.ucell, p, (c->f64 ? 8 : 4) * C, hipMemcpyHostToDevice));
    p += (c->f64 ? 8 : 4) * C;
    M2M_HIP(c, copy_sync(c->stream, c->fd.rp, p, (c->f64 ? 8 : 4) * J, hipMemcpyHostToDevice));
    p += (c->f64 ? 8 : 4) * J;
    M2M_HIP(c, copy_sync(c->stream, c->fd.chi2_hist, p, 8 * (size_t)kHistCap, hipMemcpyHostToDevice));
    p += 8 * (size_t)kHistCap;
    M2M_HIP(c, copy_sync(c->stream, c->fd.gprior, p, 8 * C, hipMemcpyHostToDevice));
    p += 8 * C;
    const size_t ST = scf_table_len(c->par);
    if (ST > 0) M2M_HIP(c, copy_sync(c->stream, c->fd.scf_tab, p, 8 * ST, hipMemcpyHostToDevice));
    c->targets = h.targets != 0;
    c->ytil_init = h.ytil_init != 0;
    return M2M_OK;
}

m2m_status m2m_profile_step(m2m_ctx* c, int32_t n_steps, int32_t correct, double* ms_step,
                            double* ms_finalize) {
    if (!c) return M2M_EINVAL;
    if (n_steps < 1 || n_steps > kProfileMax) return fail(c, M2M_EINVAL, "n_steps out of range");
    if (c->batch) return fail(c, M2M_ESTATE, "fit is in a batch");
    if (m2m_status w_ = after_batch(c); w_ != M2M_OK) return w_;
    if (!c->targets) return fail(c, M2M_ESTATE, "set targets first");
    c->may_assign = true;
    m2m_status st = ensure_graph(c);
    if (st == M2M_OK) st = ensure_prof_graph(c);
    if (st != M2M_OK) return st;
    // r replays of each graph: S per step with the plain steps, S2 with the
    // extra reduction; the reduction then costs S2 - S where it runs, and the
    // step kernel S - (S2 - S)
    const int r = (n_steps + kGraphSteps - 1) / kGraphSteps;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    hipError_t e = hipSuccess;
    for (auto& x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    if (e == hipSuccess) e = launch_poke(c->st, 2 * r * kGraphSteps, correct ? 1 : 0, c->stream);
    if (e == hipSuccess) e = hipEventRecord(ev[0], c->stream);
    for (int k = 0; k < r && e == hipSuccess; ++k) e = hipGraphLaunch(c->graph, c->stream);
    if (e == hipSuccess) e = hipEventRecord(ev[1], c->stream);
    for (int k = 0; k < r && e == hipSuccess; ++k) e = hipGraphLaunch(c->graph_prof, c->stream);
    if (e == hipSuccess) e = hipEventRecord(ev[2], c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    float t1 = 0.f, t2 = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t1, ev[0], ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&t2, ev[1], ev[2]);
    for (auto& x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess) return hip_fail(c, e, "profile");
    const double S = (double)t1 / (r * kGraphSteps), S2 = (double)t2 / (r * kGraphSteps);
    if (ms_step) *ms_step = S - (S2 - S);
    if (ms_finalize) *ms_finalize = S2 - S;
    return M2M_OK;
}

m2m_status m2m_smoothing_basis(int32_t n_E, int32_t n_x, double hE, double hx, double* out,
                               size_t* len) {
    if (!len || n_E < 1 || n_x < 1 || n_E > kSmoothMaxSide || n_x > kSmoothMaxSide ||
        n_E * n_x > kSmoothMaxCells || !(is_fin(hE) && hE > 0) || !(is_fin(hx) && hx > 0))
        return M2M_EINVAL;
    const size_t need = smooth_basis_len(n_E, n_x);
    if (!out) {
        *len = need;
        return M2M_OK;
    }
    if (*len < need) return M2M_EINVAL;
    *len = need;
    return smooth_basis(n_E, n_x, hE, hx, out) ? M2M_OK : M2M_EDEVICE;
}

m2m_status m2m_destroy(m2m_ctx* c) {
    if (!c) return M2M_EINVAL;
    if (c->batch) return fail(c, M2M_ESTATE, "fit is in a batch");
    (void)hipStreamSynchronize(c->stream);
    if (c->idle_ev) {
        // the batch runs that may still read the fit have ended
        (void)hipEventSynchronize(c->idle_ev);
        (void)hipEventDestroy(c->idle_ev);
    }
    if (c->own_ev) (void)hipEventDestroy(c->own_ev);
    if (c->graph) (void)hipGraphExecDestroy(c->graph);
    if (c->graph_prof) (void)hipGraphExecDestroy(c->graph_prof);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    if (c->own_ws) (void)hipFree(c->ws);
    delete c;
    return M2M_OK;
}

}  // extern "C"

// ================================================================= batch ===
// The tables of one launch of some fits of a batch: their descriptions, the
// tiles of the step kernel and the finalize jobs, and the graph of
// kBatchGraphSteps steps over them. A group also has a stream of its own.
struct LaunchSet {
    FitDev* fits_dev = nullptr;
    Tile* tiles_dev = nullptr;
    FinJob* jobs_dev = nullptr;
    size_t cap_fits = 0, cap_tiles = 0, cap_jobs = 0;
    int n_tiles = 0, n_jobs = 0, n_fits = 0;
    bool whole = false;  // one whole-fit finalize job per fit (else column jobs)
    bool nt = false;     // the fits' state together exceeds kStreamMin (kModeStream)
    size_t lds = 0;
    hipGraphExec_t graph = nullptr;   // kBatchGraphSteps steps
    hipStream_t stream = nullptr;  // groups: the stream the group's steps run on
    hipEvent_t done = nullptr;     // groups: the group's steps of a run call have ended
    // pinned host staging of the tables, two slots in turn: a rebuild copies
    // from one on the batch stream without waiting for the runs before it,
    // and a slot is rewritten only once its copies (two rebuilds back) ended
    unsigned char* stage[2] = {nullptr, nullptr};
    size_t stage_cap[2] = {0, 0};
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    int stage_slot = 0;
};

struct m2m_batch {
    int max_fits = 0;
    size_t budget = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;
    std::vector<m2m_ctx*> fits;
    bool dirty = true;
    int f64 = -1;
    // every fit in admission order: completion flags, timing, and the runs
    // of a batch of one fit
    LaunchSet all;
    // two groups of fits of about equal particle count, each stepping on its
    // own stream, so that one group's finalize and the tail of its step
    // kernel overlap the other group's streaming
    LaunchSet grp[kGroups];
    int n_groups = 1;
    hipEvent_t start = nullptr;  // work before a run call, which the groups wait for
    int32_t* gather_dev = nullptr;
    int32_t* gather_host = nullptr;  // pinned: the synchronous poll's flags, then two snapshots
    // completion snapshots, taken at the end of every run in two slots in
    // turn: the flags of the fits then in the batch (snap_fits; an entry
    // becomes NULL when its fit leaves the batch), and the event after them
    int32_t* snap_host[2] = {nullptr, nullptr};
    hipEvent_t snap_ev[2] = {nullptr, nullptr};
    std::vector<m2m_ctx*> snap_fits[2];
    int64_t runs = 0;       // runs enqueued
    int64_t consumed = -1;  // last run whose snapshot a lagged poll has read
    int block = 256, kin = -1;
    bool acc64 = true;
    bool smooth = false;  // some fit smooths its prior grid
    bool graphs = false;  // steps replayed from captured graphs (else launched directly)
};

namespace {

size_t footprint(const m2m_ctx* c) {
    return (size_t)c->n * 8 * (c->f64 ? 8 : 4) + c->w.total;
}

hipError_t grow(void** p, size_t* cap, size_t need) {
    if (need <= *cap) return hipSuccess;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    size_t n = std::max(need, *cap * 2);
    hipError_t e = hipMalloc(p, n);
    *cap = e == hipSuccess ? n : 0;
    return e;
}

// One batched step over a set: the step kernel over the tiles of its fits,
// then their finalize jobs.
hipError_t batch_step(const m2m_batch* b, const LaunchSet& L, bool f64, hipStream_t s) {
    hipError_t e = launch_step(f64, b->acc64, b->block, b->kin, L.fits_dev, L.tiles_dev, L.n_tiles,
                               L.lds, kModeStep | (L.nt ? kModeStream : 0), s);
    if (e == hipSuccess)
        e = launch_finalize(f64, L.fits_dev, L.n_fits, L.jobs_dev, L.n_jobs, kModeStep, s,
                            kin_scf(b->kin), b->smooth, L.whole);
    return e;
}

void free_set(LaunchSet& L) {
    if (L.graph) (void)hipGraphExecDestroy(L.graph);
    for (int k = 0; k < 2; ++k) {
        if (L.stage_ev[k]) (void)hipEventDestroy(L.stage_ev[k]);
        if (L.stage[k]) (void)hipHostFree(L.stage[k]);
        L.stage_ev[k] = nullptr;
        L.stage[k] = nullptr;
        L.stage_cap[k] = 0;
    }

    if (L.fits_dev) (void)hipFree(L.fits_dev);
    if (L.tiles_dev) (void)hipFree(L.tiles_dev);
    if (L.jobs_dev) (void)hipFree(L.jobs_dev);
    L.graph = nullptr;
    L.fits_dev = nullptr;
    L.tiles_dev = nullptr;
    L.jobs_dev = nullptr;
    L.cap_fits = L.cap_tiles = L.cap_jobs = 0;
}

// The tables of the fits `members` (indices into b->fits, in that order)
// into L, and with `capture` the graph of kBatchGraphSteps steps over them.
// One tile size for all of them, so that every block streams about the
// same number of particles; each fit's last tile may be short, so the size
// leaves one spare tile per fit: at most the launch shape's tiles in all.
m2m_status fill_set(m2m_batch* b, LaunchSet& L, const std::vector<int>& members, bool capture) {
    if (L.graph) {
        (void)hipGraphExecDestroy(L.graph);
        L.graph = nullptr;
    }
    L.n_tiles = L.n_jobs = L.n_fits = 0;
    if (members.empty()) return M2M_OK;
    const bool f64 = b->f64 == 1;
    std::vector<FitDev> fd;
    std::vector<Tile> tl;
    std::vector<FinJob> jb;
    int64_t ntot = 0;
    for (int m : members) ntot += b->fits[m]->n;
    const int target = std::max(1, g_tiles_per_cu * n_cus());
    const int64_t room = std::max<int64_t>(1, target - (int64_t)members.size());
    int64_t tile = (ntot + room - 1) / room;
    tile = (tile + kSegAlign - 1) / kSegAlign * kSegAlign;
    size_t lds = 0;
    // a launch's finalize is one block per fit when every fit's tile rows of
    // observable sums are small enough, else column jobs for every fit
    bool whole = true;
    std::vector<int> cnts(members.size());
    for (size_t f = 0; f < members.size(); ++f) {
        m2m_ctx* c = b->fits[members[f]];
        int cnt = (int)std::min<int64_t>((c->n + tile - 1) / tile, c->w.seg_cap);
        cnts[f] = std::max(1, cnt);
        if ((size_t)cnts[f] * (size_t)c->w.J * 8 > kWholeFitMaxBytes) whole = false;
    }
    for (size_t f = 0; f < members.size(); ++f) {
        m2m_ctx* c = b->fits[members[f]];
        fd.push_back(c->fd);
        split_tiles(c->n, cnts[f], (int)f, 0, tl);
        if (whole)
            jb.push_back(FinJob{(int)f, kFinWholeFit, 0, cnts[f]});
        else
            fin_jobs(c->w, (int)f, cnts[f], jb);
        lds = std::max(lds, c->lds);
    }
    const size_t bf = sizeof(FitDev) * fd.size(), bt = sizeof(Tile) * tl.size(),
                 bj = sizeof(FinJob) * jb.size();
    if (bf > L.cap_fits || bt > L.cap_tiles || bj > L.cap_jobs) {
        // larger device tables (rare): the old ones are freed only after
        // every run that reads them has ended (the groups' work joins the
        // batch stream at the end of every run)
        if (hipStreamSynchronize(b->stream) != hipSuccess) return M2M_EDEVICE;
        if (grow(reinterpret_cast<void**>(&L.fits_dev), &L.cap_fits, bf) != hipSuccess ||
            grow(reinterpret_cast<void**>(&L.tiles_dev), &L.cap_tiles, bt) != hipSuccess ||
            grow(reinterpret_cast<void**>(&L.jobs_dev), &L.cap_jobs, bj) != hipSuccess)
            return M2M_ENOMEM;
    }
    // the tables through a pinned staging slot, copied on the batch stream:
    // after the runs already enqueued (which still read the old tables) and
    // before the next one, without the host waiting for either
    const int sl = L.stage_slot;
    L.stage_slot ^= 1;
    if (L.stage_ev[sl] && hipEventSynchronize(L.stage_ev[sl]) != hipSuccess) return M2M_EDEVICE;
    if (!L.stage_ev[sl] && hipEventCreateWithFlags(&L.stage_ev[sl], hipEventDisableTiming) != hipSuccess)
        return M2M_EDEVICE;
    if (bf + bt + bj > L.stage_cap[sl]) {
        if (L.stage[sl]) (void)hipHostFree(L.stage[sl]);
        L.stage[sl] = nullptr;
        const size_t cap = std::max(bf + bt + bj, 2 * L.stage_cap[sl]);
        L.stage_cap[sl] = 0;
        if (hipHostMalloc(reinterpret_cast<void**>(&L.stage[sl]), cap, 0) != hipSuccess) return M2M_ENOMEM;
        L.stage_cap[sl] = cap;
    }
    unsigned char* st = L.stage[sl];
    std::memcpy(st, fd.data(), bf);
    std::memcpy(st + bf, tl.data(), bt);
    std::memcpy(st + bf + bt, jb.data(), bj);
    if (hipMemcpyAsync(L.fits_dev, st, bf, hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipMemcpyAsync(L.tiles_dev, st + bf, bt, hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipMemcpyAsync(L.jobs_dev, st + bf + bt, bj, hipMemcpyHostToDevice, b->stream) != hipSuccess ||
        hipEventRecord(L.stage_ev[sl], b->stream) != hipSuccess)
        return M2M_EDEVICE;
    L.n_tiles = (int)tl.size();
    L.n_jobs = (int)jb.size();
    L.n_fits = (int)fd.size();
    L.whole = whole;
    size_t state = 0;
    for (int m : members) state += (size_t)b->fits[m]->n * 8 * (f64 ? 8 : 4);
    L.nt = state > kStreamMin;
    L.lds = lds;
    if (capture) {
        // the graph of kBatchGraphSteps steps, uploaded on the stream it
        // will run on
        const LaunchSet* Lp = &L;
        auto body = [b, Lp, f64](hipStream_t s) { return batch_step(b, *Lp, f64, s); };
        hipStream_t up = L.stream ? L.stream : b->stream;
        if (capture_steps(b->cap, kBatchGraphSteps, body, &L.graph, up) != hipSuccess)
            return M2M_EDEVICE;
    }
    return M2M_OK;
}

m2m_status rebuild(m2m_batch* b) {
    // graphs in flight cannot be replaced under them: with graphs, wait for
    // the runs enqueued (the groups' work joins the batch stream at the end
    // of every run); without, the new tables are copied in stream order
    const bool graphs = b->all.graph || b->grp[0].graph || b->grp[1].graph || g_batch_graphs;
    if (graphs && hipStreamSynchronize(b->stream) != hipSuccess) return M2M_EDEVICE;
    const int nf = (int)b->fits.size();
    b->n_groups = nf >= 2 ? g_groups : 1;
    if (nf == 0) {
        for (LaunchSet* L : {&b->all, &b->grp[0], &b->grp[1]}) {
            if (L->graph) (void)hipGraphExecDestroy(L->graph);
            L->graph = nullptr;
            L->n_tiles = L->n_jobs = L->n_fits = 0;
        }
        b->dirty = false;
        return M2M_OK;
    }
    b->block = b->f64 == 1 ? 256 : g_block;
    b->acc64 = b->f64 == 1 || g_deposit == M2M_DEPOSIT_F64;
    b->smooth = false;
    for (m2m_ctx* c : b->fits)
        if (c->par.smooth) b->smooth = true;
    std::vector<int> every(nf);
    for (int f = 0; f < nf; ++f) every[f] = f;
    b->graphs = g_batch_graphs != 0;
    m2m_status s = fill_set(b, b->all, every, b->graphs && b->n_groups == 1);
    if (s != M2M_OK) return s;
    if (b->n_groups > 1) {
        // the largest fits first, each to the group with fewer particles
        std::vector<int> order = every;
        std::stable_sort(order.begin(), order.end(),
                         [b](int x, int y) { return b->fits[x]->n > b->fits[y]->n; });
        std::vector<int> mem[kGroups];
        int64_t load[kGroups] = {0, 0};
        for (int f : order) {
            const int g = load[1] < load[0] ? 1 : 0;
            mem[g].push_back(f);
            load[g] += b->fits[f]->n;
        }
        for (int g = 0; g < kGroups; ++g) {
            std::sort(mem[g].begin(), mem[g].end());
            if ((s = fill_set(b, b->grp[g], mem[g], b->graphs)) != M2M_OK) return s;
        }
    }
    b->dirty = false;
    return M2M_OK;
}

// steps of the set L on stream st: with graphs, graphs of kBatchGraphSteps
// steps and then direct launches (a graph launch has a fixed cost of several
// kernel launches); without, direct launches only
hipError_t run_set(const m2m_batch* b, const LaunchSet& L, int steps, hipStream_t st) {
    const bool f64 = b->f64 == 1;
    const int full = L.graph ? steps / kBatchGraphSteps : 0;
    hipError_t e = hipSuccess;
    for (int k = 0; k < full && e == hipSuccess; ++k) e = hipGraphLaunch(L.graph, st);
    for (int k = full * kBatchGraphSteps; k < steps && e == hipSuccess; ++k)
        e = batch_step(b, L, f64, st);
    return e;
}

// The fit leaves the batch: its idle event is recorded after every run
// enqueued so far (the last of them may still read it), and the snapshots
// forget it, so that no later poll reads the context.
hipError_t retire(m2m_batch* b, m2m_ctx* c) {
    c->batch = nullptr;
    c->may_assign = true;  // its batched steps may have refreshed the priors
    for (auto& v : b->snap_fits)
        for (m2m_ctx*& x : v)
            if (x == c) x = nullptr;
    hipError_t e = hipSuccess;
    if (!c->idle_ev) e = hipEventCreateWithFlags(&c->idle_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(c->idle_ev, b->stream);
    c->idle_pending = e == hipSuccess;
    return e;
}

// The completion flags of the fits in the batch, taken on the batch stream
// at the end of a run into the run's snapshot slot.
hipError_t snapshot(m2m_batch* b) {
    const int nf = (int)b->fits.size();
    const int sl = (int)(b->runs & 1);
    hipError_t e = hipSuccess;
    if (nf > 0) {
        e = launch_gather(b->all.fits_dev, nf, b->gather_dev, b->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->snap_host[sl], b->gather_dev, sizeof(int32_t) * 2 * nf,
                               hipMemcpyDeviceToHost, b->stream);
    }
    if (e == hipSuccess) e = hipEventRecord(b->snap_ev[sl], b->stream);
    b->snap_fits[sl] = b->fits;
    ++b->runs;
    return e;
}

// Hands back up to max_done of `fits` that have no steps left by their flags
// (steps left and error bits, two per fit; NULL entries and fits no longer
// in the batch are skipped) and takes them out of the batch.
m2m_status collect(m2m_batch* b, const std::vector<m2m_ctx*>& fits, const int32_t* flags,
                   m2m_ctx** done, int32_t max_done, int32_t* n_done) {
    std::vector<m2m_ctx*> gone;
    bool bad = false;
    for (size_t f = 0; f < fits.size() && *n_done < max_done; ++f) {
        m2m_ctx* c = fits[f];
        if (!c || c->batch != b || flags[2 * f] > 0) continue;
        done[(*n_done)++] = c;
        gone.push_back(c);
        if (flags[2 * f + 1] & 1) {
            c->err = "chi^2 became non-finite";
            bad = true;
        }
    }
    bool dev = false;
    for (m2m_ctx* c : gone) {
        b->fits.erase(std::find(b->fits.begin(), b->fits.end(), c));
        if (retire(b, c) != hipSuccess) dev = true;
    }
    if (!gone.empty()) {
        b->dirty = true;
        if (b->fits.empty()) b->f64 = -1;
    }
    return dev ? M2M_EDEVICE : (bad ? M2M_ENONFINITE : M2M_OK);
}

}  // namespace

extern "C" {

m2m_status m2m_batch_create(int32_t max_fits, size_t hbm_budget, void* hip_stream,
                            m2m_batch** out) {
    if (!out) return M2M_EINVAL;
    *out = nullptr;
    if (max_fits < 1 || max_fits > 65536) return M2M_EINVAL;
    m2m_batch* b = new (std::nothrow) m2m_batch();
    if (!b) return M2M_ENOMEM;
    b->max_fits = max_fits;
    b->budget = hbm_budget;
    b->stream = static_cast<hipStream_t>(hip_stream);
    bool ok = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&b->start, hipEventDisableTiming) == hipSuccess;
    for (int g = 0; g < kGroups && ok; ++g)
        ok = hipStreamCreateWithFlags(&b->grp[g].stream, hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&b->grp[g].done, hipEventDisableTiming) == hipSuccess;
    ok = ok && hipMalloc(reinterpret_cast<void**>(&b->gather_dev), sizeof(int32_t) * 2 * (size_t)max_fits) == hipSuccess &&
         hipHostMalloc(reinterpret_cast<void**>(&b->gather_host), sizeof(int32_t) * 6 * (size_t)max_fits, 0) == hipSuccess;
    for (int k = 0; k < 2 && ok; ++k) {
        b->snap_host[k] = b->gather_host + 2 * (size_t)max_fits * (k + 1);
        ok = hipEventCreateWithFlags(&b->snap_ev[k], hipEventDisableTiming) == hipSuccess;
    }
    if (!ok) {
        (void)m2m_batch_destroy(b);
        return M2M_EDEVICE;
    }
    *out = b;
    return M2M_OK;
}

size_t m2m_batch_footprint(const m2m_batch* b) {
    if (!b) return 0;
    size_t s = 0;
    for (const m2m_ctx* c : b->fits) s += footprint(c);
    return s;
}

m2m_status m2m_batch_admit(m2m_batch* b, m2m_ctx* c, int32_t n_steps) {
    if (!b || !c || n_steps < 0) return M2M_EINVAL;
    if (c->batch) return fail(c, M2M_ESTATE, "fit is already in a batch");
    if (!c->targets) return fail(c, M2M_ESTATE, "set targets first");
    if (b->f64 != -1 && b->f64 != (c->f64 ? 1 : 0))
        return fail(c, M2M_EINVAL, "a batch holds fits of one particle dtype");
    if (!b->fits.empty() && b->kin != c->kin)
        return fail(c, M2M_EINVAL, "a batch holds fits of one kind of kinematic observable");
    if ((int)b->fits.size() >= b->max_fits) return fail(c, M2M_ENOMEM, "batch is full");
    if (b->budget && m2m_batch_footprint(b) + footprint(c) > b->budget)
        return fail(c, M2M_ENOMEM, "fit does not fit the HBM budget");
    m2m_status s = after_batch(c);
    if (s != M2M_OK) return s;
    if ((s = flush_assign(c)) != M2M_OK) return s;
    // the batch stream waits for the fit's own work (its creation, targets,
    // steps) on the device; the host does not wait
    if (!c->own_ev) M2M_HIP(c, hipEventCreateWithFlags(&c->own_ev, hipEventDisableTiming));
    M2M_HIP(c, hipEventRecord(c->own_ev, c->stream));
    M2M_HIP(c, hipStreamWaitEvent(b->stream, c->own_ev, 0));
    M2M_HIP(c, launch_poke(c->st, n_steps, 1, b->stream));
    b->f64 = c->f64 ? 1 : 0;
    b->kin = c->kin;
    b->fits.push_back(c);
    c->batch = b;
    b->dirty = true;
    return M2M_OK;
}

m2m_status m2m_batch_run(m2m_batch* b, int32_t steps_per_launch) {
    if (!b || steps_per_launch < 0) return M2M_EINVAL;
    if (b->dirty) {
        m2m_status s = rebuild(b);
        if (s != M2M_OK) return s;
    }
    if (b->fits.empty() || steps_per_launch == 0) return M2M_OK;
    if (b->n_groups == 1) {
        hipError_t e = run_set(b, b->all, steps_per_launch, b->stream);
        if (e == hipSuccess) e = snapshot(b);
        return e == hipSuccess ? M2M_OK : M2M_EDEVICE;
    }
    // the groups start after the work already on the batch stream, and the
    // batch stream continues after both; their steps are enqueued in turn
    // (step k of every group, then step k + 1), as the runtime blocks the
    // host once a stream has many launches outstanding, and a group enqueued
    // whole before the other would run alone meanwhile
    hipError_t e = hipEventRecord(b->start, b->stream);
    for (int g = 0; g < b->n_groups && e == hipSuccess; ++g)
        e = hipStreamWaitEvent(b->grp[g].stream, b->start, 0);
    const bool f64 = b->f64 == 1;
    const int full = b->graphs ? steps_per_launch / kBatchGraphSteps : 0;
    for (int k = 0; k < full && e == hipSuccess; ++k)
        for (int g = 0; g < b->n_groups && e == hipSuccess; ++g)
            e = hipGraphLaunch(b->grp[g].graph, b->grp[g].stream);
    for (int k = full * kBatchGraphSteps; k < steps_per_launch && e == hipSuccess; ++k)
        for (int g = 0; g < b->n_groups && e == hipSuccess; ++g)
            e = batch_step(b, b->grp[g], f64, b->grp[g].stream);
    for (int g = 0; g < b->n_groups && e == hipSuccess; ++g)
        e = hipEventRecord(b->grp[g].done, b->grp[g].stream);
    for (int g = 0; g < b->n_groups && e == hipSuccess; ++g)
        e = hipStreamWaitEvent(b->stream, b->grp[g].done, 0);
    if (e == hipSuccess) e = snapshot(b);
    return e == hipSuccess ? M2M_OK : M2M_EDEVICE;
}

m2m_status m2m_batch_poll(m2m_batch* b, m2m_ctx** done, int32_t max_done, int32_t* n_done,
                          int32_t* n_active) {
    if (!b || !n_done || max_done < 0 || (max_done > 0 && !done)) return M2M_EINVAL;
    *n_done = 0;
    if (b->dirty) {
        m2m_status s = rebuild(b);
        if (s != M2M_OK) return s;
    }
    const int nf = (int)b->fits.size();
    if (nf > 0) {
        if (launch_gather(b->all.fits_dev, nf, b->gather_dev, b->stream) != hipSuccess ||
            hipMemcpyAsync(b->gather_host, b->gather_dev, sizeof(int32_t) * 2 * nf,
                           hipMemcpyDeviceToHost, b->stream) != hipSuccess)
            return M2M_EDEVICE;
    }
    if (hipStreamSynchronize(b->stream) != hipSuccess) return M2M_EDEVICE;
    const std::vector<m2m_ctx*> now = b->fits;
    const m2m_status s = collect(b, now, b->gather_host, done, max_done, n_done);
    if (n_active) *n_active = (int32_t)b->fits.size();
    return s;
}

m2m_status m2m_batch_poll_lagged(m2m_batch* b, m2m_ctx** done, int32_t max_done,
                                 int32_t* n_done, int32_t* n_active) {
    if (!b || !n_done || max_done < 0 || (max_done > 0 && !done)) return M2M_EINVAL;
    *n_done = 0;
    // the run before the latest: its snapshot slot is not rewritten before
    // the next run, and the latest run keeps the device busy meanwhile
    const int64_t k = b->runs - 2;
    m2m_status s = M2M_OK;
    if (k >= 0 && k > b->consumed) {
        const int sl = (int)(k & 1);
        if (hipEventSynchronize(b->snap_ev[sl]) != hipSuccess) return M2M_EDEVICE;
        b->consumed = k;
        s = collect(b, b->snap_fits[sl], b->snap_host[sl], done, max_done, n_done);
    }
    if (n_active) *n_active = (int32_t)b->fits.size();
    return s;
}

m2m_status m2m_batch_profile(m2m_batch* b, int32_t n_steps, double* ms_step, double* ms_finalize) {
    if (!b || n_steps < 1 || n_steps > kBatchProfileMax) return M2M_EINVAL;
    if (b->dirty) {
        m2m_status s = rebuild(b);
        if (s != M2M_OK) return s;
    }
    if (b->fits.empty()) return M2M_ESTATE;
    // n_steps steps of all fits launched one kernel at a time (one step
    // kernel over the tiles of every fit, not the overlapping groups), each
    // step kernel between two events on the batch stream: its duration (with
    // the events' own small cost, so an upper bound), and the rest of the
    // step (the finalize and the gaps) from its second event to the next
    // step's first
    const bool f64 = b->f64 == 1;
    std::vector<hipEvent_t> ev(2 * (size_t)n_steps + 1, nullptr);
    hipError_t e = hipSuccess;
    for (auto& x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    for (int k = 0; k < n_steps && e == hipSuccess; ++k) {
        e = hipEventRecord(ev[2 * k], b->stream);
        if (e == hipSuccess)
            e = launch_step(f64, b->acc64, b->block, b->kin, b->all.fits_dev, b->all.tiles_dev,
                            b->all.n_tiles, b->all.lds, kModeStep | (b->all.nt ? kModeStream : 0),
                            b->stream);
        if (e == hipSuccess) e = hipEventRecord(ev[2 * k + 1], b->stream);
        if (e == hipSuccess)
            e = launch_finalize(f64, b->all.fits_dev, b->all.n_fits, b->all.jobs_dev, b->all.n_jobs,
                                kModeStep, b->stream, kin_scf(b->kin), b->smooth, b->all.whole);
    }
    if (e == hipSuccess) e = hipEventRecord(ev[2 * (size_t)n_steps], b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    double ts = 0.0, tf = 0.0;
    for (int k = 0; k < n_steps && e == hipSuccess; ++k) {
        float a = 0.f, c = 0.f;
        e = hipEventElapsedTime(&a, ev[2 * k], ev[2 * k + 1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&c, ev[2 * k + 1], ev[2 * k + 2]);
        ts += a;
        tf += c;
    }
    for (auto& x : ev)
        if (x) (void)hipEventDestroy(x);
    if (e != hipSuccess) return M2M_EDEVICE;
    if (ms_step) *ms_step = ts / n_steps;
    if (ms_finalize) *ms_finalize = tf / n_steps;
    return M2M_OK;
}

int64_t m2m_batch_particles(m2m_batch* b) {
    if (!b) return 0;
    const int nf = (int)b->fits.size();
    if (nf == 0) return 0;
    if (b->dirty && rebuild(b) != M2M_OK) return -1;
    if (launch_gather(b->all.fits_dev, nf, b->gather_dev, b->stream) != hipSuccess ||
        hipMemcpyAsync(b->gather_host, b->gather_dev, sizeof(int32_t) * 2 * nf,
                       hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
        return -1;
    int64_t n = 0;
    for (int f = 0; f < nf; ++f)
        if (b->gather_host[2 * f] > 0) n += b->fits[f]->n;
    return n;
}

m2m_status m2m_batch_cancel(m2m_batch* b, m2m_ctx* c) {
    if (!b || !c || c->batch != b) return M2M_EINVAL;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return M2M_EDEVICE;
    if (launch_poke(c->st, 0, -1, b->stream) != hipSuccess ||
        hipStreamSynchronize(b->stream) != hipSuccess)
        return M2M_EDEVICE;
    b->fits.erase(std::find(b->fits.begin(), b->fits.end(), c));
    const hipError_t e = retire(b, c);
    b->dirty = true;
    if (b->fits.empty()) b->f64 = -1;
    return e == hipSuccess ? M2M_OK : M2M_EDEVICE;
}

m2m_status m2m_batch_destroy(m2m_batch* b) {
    if (!b) return M2M_EINVAL;
    (void)hipStreamSynchronize(b->stream);
    for (m2m_ctx* c : b->fits) c->batch = nullptr;
    free_set(b->all);
    for (int g = 0; g < kGroups; ++g) {
        free_set(b->grp[g]);
        if (b->grp[g].stream) (void)hipStreamDestroy(b->grp[g].stream);
        if (b->grp[g].done) (void)hipEventDestroy(b->grp[g].done);
    }
    if (b->start) (void)hipEventDestroy(b->start);
    for (hipEvent_t x : b->snap_ev)
        if (x) (void)hipEventDestroy(x);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->gather_dev) (void)hipFree(b->gather_dev);
    if (b->gather_host) (void)hipHostFree(b->gather_host);
    delete b;
    return M2M_OK;
}

}  // extern "C"

// ================================================ allocation-free observe ==
// The working memory of m2m_observe_noalloc: a static device array, one copy
// per GPU at its own address. Host code never passes the array's name to a
// kernel or a copy (on the host it stands for no device address): the
// address is looked up once per device with hipGetSymbolAddress, with that
// device current, and kept in g_na_ptr.
static __device__ __align__(256) unsigned char scratch[M2M_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kNoAllocDevices = 64;
constexpr size_t kNoAllocStage = (size_t)256 << 10;  // host image of the tables
std::mutex g_na_mu;                        // one call at a time in a process
void* g_na_ptr[kNoAllocDevices];           // address of `scratch` per device
unsigned char g_na_stage[kNoAllocStage];   // staging of the tables (under g_na_mu)

m2m_status na_fail(m2m_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_na_err, sizeof g_na_err, fmt, ap);
    va_end(ap);
    return s;
}
}  // namespace

extern "C" m2m_status m2m_observe_noalloc(const m2m_obs_layout* layout, double mass, int64_t n,
                                          int32_t dtype, const void* x, const void* y,
                                          const void* z, const void* vx, const void* vy,
                                          const void* vz, const void* u, const double* V_p,
                                          const double* sigma_p, double* obs, void* hip_stream) {
    g_na_err[0] = '\0';
    if (!layout) return na_fail(M2M_EINVAL, "layout is NULL");
    {
        const std::string why = check_layout(layout);
        if (!why.empty()) return na_fail(M2M_EINVAL, "%s", why.c_str());
    }
    if (!(is_fin(mass) && mass > 0)) return na_fail(M2M_EINVAL, "mass must be finite and > 0");
    if (n < 1) return na_fail(M2M_EINVAL, "n must be >= 1");
    if (dtype != M2M_F32 && dtype != M2M_F64) return na_fail(M2M_EINVAL, "unknown dtype");
    const void* const ptrs[7] = {x, y, z, vx, vy, vz, u};
    for (const void* q : ptrs)
        if (!q || (reinterpret_cast<uintptr_t>(q) & 15u))
            return na_fail(M2M_EINVAL, "particle arrays must be non-NULL and 16-byte aligned");
    if (!obs) return na_fail(M2M_EINVAL, "obs is NULL");
    const m2m_obs_layout& L = *layout;
    const int nR = L.kin == M2M_KIN_NONE ? 0 : L.n_R;
    if (L.kin == M2M_KIN_GH) {
        if (!V_p || !sigma_p)
            return na_fail(M2M_EINVAL, "Gauss-Hermite observables need V_p and sigma_p");
        for (int q = 0; q < nR; ++q)
            if (!is_fin(V_p[q]) || !is_fin(sigma_p[q]) || !(sigma_p[q] > 0))
                return na_fail(M2M_EINVAL, "V_p, sigma_p must be finite with sigma_p > 0");
    }
    const bool f64 = dtype == M2M_F64;
    // observation only: one prior cell, no smoothing, no self-consistent
    // potential, no per-particle cell index
    m2m_params P{};
    P.mass = mass;
    P.n_E = 1;
    P.n_x = 1;
    P.E_lo = -1.0;
    P.E_hi = 0.0;
    const WsLayout w = plan(L, P, n, f64, false);
    if (w.total > (size_t)M2M_NOALLOC_SCRATCH_BYTES)
        return na_fail(M2M_ENOMEM,
                       "observation needs %zu bytes of working memory, more than the %zu bytes "
                       "of the static scratch",
                       w.total, (size_t)M2M_NOALLOC_SCRATCH_BYTES);
    if (w.rp - w.redge2 > kNoAllocStage)
        return na_fail(M2M_ENOMEM, "observation tables exceed the %zu-byte staging area",
                       kNoAllocStage);
    const int kpriv = g_kpriv_cap > 0 ? std::min(private_copies(f64, w.J), g_kpriv_cap)
                                      : private_copies(f64, w.J);
    const bool acc64 = f64 || g_deposit == M2M_DEPOSIT_F64;
    const size_t lds = step_lds_bytes(f64, acc64, w.J, radial_intervals(L), nR,
                                      L.kin == M2M_KIN_LOSVD ? L.n_v : 0, kpriv, w.C, 0, 0);
    if (lds > max_lds()) return na_fail(M2M_EUNSUPPORTED, "the observable bins do not fit LDS");
    const int block = f64 ? 256 : g_block;
    const int kin = kin_class(L.kin, L.gh_nmax, L.dens, false);
    // the tiles of a context of the same particle count (m2m_create)
    const int n_tiles = std::max(1, std::min(w.seg_cap, std::max(1, g_tiles_per_cu * n_cus())));

    std::lock_guard<std::mutex> lock(g_na_mu);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return na_fail(M2M_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kNoAllocDevices)
        return na_fail(M2M_EUNSUPPORTED, "device %d: at most %d devices", dev, kNoAllocDevices);
    if (!g_na_ptr[dev]) {
        void* q = nullptr;
        e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !q)
            return na_fail(M2M_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_na_ptr[dev] = q;
    }
    unsigned char* b = static_cast<unsigned char*>(g_na_ptr[dev]);

    FitDev f{};
    f.x = const_cast<void*>(x);
    f.y = const_cast<void*>(y);
    f.z = const_cast<void*>(z);
    f.vx = const_cast<void*>(vx);
    f.vy = const_cast<void*>(vy);
    f.vz = const_cast<void*>(vz);
    f.u = const_cast<void*>(u);
    f.uh = const_cast<void*>(u);  // priors: never read when observing
    f.n = n;
    f.w0 = mass / (double)n;
    f.a = 1.0;
    f.rs = 1.0;
    f.scf_every = 1;
    f.n_E = 1;
    f.n_x = 1;
    f.cell_half = 1;
    describe_obs(f, L, w, b);
    f.kpriv = kpriv;
    put_obs_tables(g_na_stage, w, L, f64, V_p, sigma_p);
    // the fit's counters start at zero (the observation's ticket among them)
    static const FitState zero_state{};
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if ((e = hipMemcpyAsync(b + w.st, &zero_state, sizeof(FitState), hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(b + w.redge2, g_na_stage, w.rp - w.redge2, hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = launch_step1(f64, acc64, block, kin, f, n_tiles, lds, kModeObserve, s)) != hipSuccess ||
        (e = launch_finalize1(f64, f, n_tiles, kModeObserve, s)) != hipSuccess ||
        (e = hipMemcpyAsync(obs, b + w.obs, 8 * (size_t)w.J, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return na_fail(M2M_EDEVICE, "observation: %s", hipGetErrorString(e));
    return M2M_OK;
}

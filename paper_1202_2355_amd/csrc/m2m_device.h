// Device helpers shared by the HIP kernels of the M2M step: global-memory
// views, elementary functions, LDS tables, per-tile constants, binning,
// spherical harmonics, the potential and the in-tile accumulation.
// Included by m2m_kernels.hip and by the step-kernel units.
#pragma once

#include <hip/hip_runtime.h>

#include "m2m_internal.h"

namespace m2m {
namespace {

// ------------------------------------------------------------- memory ------
// Device arrays reached through pointers stored in the fit table are seen
// through the global address space: accesses compile to global (not flat)
// loads and stores, which do not also wait on the LDS counter, so loads in
// flight overlap the LDS work of the particle loop.
template <typename T>
using G = __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ G<T> gmem(T* p) {
    return (G<T>)p;
}

template <typename T>
__device__ __forceinline__ G<T> gmem(void* p) {
    return (G<T>)static_cast<T*>(p);
}

// ------------------------------------------------------------- math --------
// FP32: the hardware transcendental and reciprocal instructions (about 1 ulp;
// arguments here are never denormal). FP64: the correctly rounded library.
template <typename T>
struct Mth;

template <>
struct Mth<float> {
    __device__ static float exp_(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }
    __device__ static float log_(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
    __device__ static float log2_(float x) { return __builtin_amdgcn_logf(x); }
    __device__ static float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    // log(1 + x) by Goldberg's method (What every computer scientist should
    // know about floating-point arithmetic, 1991): with u = 1 + x rounded,
    // x log(u) / (u - 1), where u - 1 is exact; x itself when u = 1
    __device__ static float log1p_(float x) {
        const float u = 1.0f + x;
        return u == 1.0f ? x : x * (log_(u) * rcp_(u - 1.0f));
    }
    __device__ static float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
    static constexpr float nfw_series_max = 0.1f;
    static constexpr float max_ = 3.40282347e38f;  // largest finite value
};

template <>
struct Mth<double> {
    __device__ static double exp_(double x) { return exp(x); }
    __device__ static double log_(double x) { return log(x); }
    __device__ static double log2_(double x) { return log2(x); }
    __device__ static double sqrt_(double x) { return sqrt(x); }
    __device__ static double log1p_(double x) { return log1p(x); }
    __device__ static double rcp_(double x) { return 1.0 / x; }
    static constexpr double nfw_series_max = 1e-3;
    static constexpr double max_ = 1.7976931348623157e308;
};

// normalized Hermite recurrence coefficients: H_{n+1} = a_n nu H_n - b_n H_{n-1}
// with a_n = sqrt(2/(n+1)), b_n = sqrt(n/(n+1)), n = 1..7
__constant__ double kGhA[kMaxGH] = {0.0,
                                   1.0,                   // sqrt(2/2)
                                   0.81649658092772603,   // sqrt(2/3)
                                   0.70710678118654752,   // sqrt(2/4)
                                   0.63245553203367587,   // sqrt(2/5)
                                   0.57735026918962576,   // sqrt(2/6)
                                   0.53452248382484880,   // sqrt(2/7)
                                   0.5};                  // sqrt(2/8)
__constant__ double kGhB[kMaxGH] = {0.0,
                                   0.70710678118654752,   // sqrt(1/2)
                                   0.81649658092772603,   // sqrt(2/3)
                                   0.86602540378443865,   // sqrt(3/4)
                                   0.89442719099991588,   // sqrt(4/5)
                                   0.91287092917527690,   // sqrt(5/6)
                                   0.92582009977255146,   // sqrt(6/7)
                                   0.93541434669348535};  // sqrt(7/8)

// ------------------------------------------------------------- LDS ---------
// In-tile bins: FP64 sums (A = double), or FP32 sums with an FP32 array of
// their compensation (A = float). They are kept in kpriv private copies,
// interleaved (copy g of bin j at j * kpriv + g); lane l adds into copy
// l mod kpriv. Then the prior-cell sums of the tile (FP64 weight sums and
// integer counts), then the tables. The 8-byte arrays come first so that
// they are aligned.
template <typename T, typename A>
struct Tabs {
    A *sum, *comp;
    double* csum;
    uint32_t* ccnt;
    T *rp, *re2, *Re2, *ve, *Vp, *isp, *rm;
    unsigned char* end;  // first byte after the tables
};

template <typename T, typename A>
__device__ __forceinline__ Tabs<T, A> carve(unsigned char* raw, int J, int kp, int n_r, int n_R,
                                            int n_v, int C) {
    Tabs<T, A> t;
    A* q = reinterpret_cast<A*>(raw);
    t.sum = q;
    q += J * kp;
    t.comp = q;
    if (sizeof(A) == 4) q += J * kp;
    t.csum = reinterpret_cast<double*>(q);
    t.ccnt = reinterpret_cast<uint32_t*>(t.csum + C);
    T* p = reinterpret_cast<T*>(t.ccnt + ((C + 1) & ~1));  // 8-byte aligned
    t.rp = p;
    p += J;
    t.re2 = p;
    p += n_r + 1;
    t.Re2 = p;
    p += n_R + 1;
    t.ve = p;
    p += n_v + 1;
    t.Vp = p;
    p += n_R;
    t.isp = p;
    p += n_R;
    t.rm = p;  // a_lm mesh radii (n_r + 1)
    t.end = reinterpret_cast<unsigned char*>(p + n_r + 1);
    return t;
}

// ------------------------------------------------------------- per tile ----
// What the particle loop reads of its fit, loaded once per tile (uniform
// values) instead of from the fit table inside the loop.
template <typename T>
struct Hot {
    int n_r, n_R, nk, gh_nmax, n_v, J, C, kp, n_E, n_x;
    int jk0, l_max, nlm;  // first kinematic observable; a_lm degree and (l_max + 1)^2
    T lr0, lrs, lR0, lRs, vmin, vidv;
    T r2lo, r2hi, R2lo, R2hi, vlo, vhi;  // range ends: squared radii, velocities
    T GMh, a, GMn, rs, irs, phi0;
    T dt, hdt, w0, foc_mu, foc_cs;
    T E_lo, E_scale, lz0, ilz;  // E_lo, E_scale: offset and scale of the cells' energy coordinate
    int cell_flags, cell_half;
    int halo;                // logarithmic halo present
    T hv2, hr02, hiq2, iv2;  // its v0^2, r0^2, 1/q^2 and 1/v0^2
    G<const T> lctab;
};

template <typename T>
__device__ __forceinline__ Hot<T> hot_of(const FitDev& fd) {
    Hot<T> h;
    h.n_r = fd.n_r;
    h.n_R = fd.n_R;
    h.nk = fd.nk;
    h.gh_nmax = fd.gh_nmax;
    h.n_v = fd.n_v;
    h.J = fd.J;
    h.C = fd.C;
    h.kp = fd.kpriv;
    h.n_E = fd.n_E;
    h.n_x = fd.n_x;
    h.jk0 = fd.jk0;
    h.l_max = fd.l_max;
    h.nlm = (fd.l_max + 1) * (fd.l_max + 1);
    h.lr0 = T(fd.lr0);
    h.lrs = T(fd.lrs);
    h.lR0 = T(fd.lR0);
    h.lRs = T(fd.lRs);
    h.vmin = T(fd.vmin);
    h.vidv = T(fd.vidv);
    const G<const T> re2 = gmem<const T>(fd.redge2);
    const G<const T> Re2 = gmem<const T>(fd.Redge2);
    const G<const T> ve = gmem<const T>(fd.vedge);
    h.r2lo = re2[0];
    h.r2hi = re2[fd.n_r];
    h.R2lo = Re2[0];
    h.R2hi = Re2[fd.n_R];
    h.vlo = ve[0];
    h.vhi = ve[fd.n_v];
    h.GMh = T(fd.GMh);
    h.a = T(fd.a);
    h.GMn = T(fd.GMn);
    h.rs = T(fd.rs);
    h.irs = T(1.0 / fd.rs);
    h.phi0 = T(fd.phi0);
    h.dt = T(fd.dt);
    h.hdt = T(0.5 * fd.dt);
    h.w0 = T(fd.w0);
    h.foc_mu = T(fd.foc_mu);
    h.foc_cs = T(fd.foc_cs);
    h.E_lo = T(fd.cell_e0);
    h.E_scale = T(fd.cell_es);
    h.cell_flags = fd.cell_flags;
    h.cell_half = fd.cell_half;
    h.halo = fd.hv2 > 0.0;
    h.hv2 = T(fd.hv2);
    h.hr02 = T(fd.hr02);
    h.hiq2 = T(fd.hiq2);
    h.iv2 = T(fd.hv2 > 0.0 ? 1.0 / fd.hv2 : 0.0);
    h.lz0 = T(fd.lz0);
    h.ilz = T(fd.ilz);
    h.lctab = gmem<const T>(fd.lctab);
    return h;
}

// ------------------------------------------------------------- binning -----
// k with e[k] <= v < e[k+1] for ascending e[0..n], decided by comparison with
// the stored edges (v is known to lie in [e[0], e[n])).
template <typename T>
__device__ __forceinline__ int refine_bin(T v, const T* e, int n, T g) {
    g = fmin(fmax(g, T(0)), T(n - 1));
    int k = (int)g;
    if (v < e[k]) {
        --k;
        if (k > 0 && v < e[k]) --k;
    } else if (v >= e[k + 1]) {
        ++k;
        if (k < n - 1 && v >= e[k + 1]) ++k;
    }
    if (!(v >= e[k] && v < e[k + 1])) {  // the guess was off by more than 2
        int lo = 0, hi = n;               // invariant e[lo] <= v < e[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (v >= e[mid]) lo = mid; else hi = mid;
        }
        k = lo;
    }
    return k;
}

// Bin of v, or -1 outside [lo, hi). The arithmetic position g of v in bin
// units is accurate to a few 1e-6, so a point more than 1e-4 of a bin from
// both edges is in bin floor(g); only points closer to an edge are compared
// with the stored edges.
template <typename T>
__device__ __forceinline__ int bin_of(T v, const T* e, int n, T g, T lo, T hi) {
    if (!(v >= lo) || !(v < hi)) return -1;
    const T gc = fmin(fmax(g, T(0)), T(n));
    const int k = min((int)gc, n - 1);
    const T fr = g - T(k);
    if (fr > T(1e-4) && fr < T(1) - T(1e-4)) return k;
    return refine_bin<T>(v, e, n, g);
}

// kinds of kinematic observables, fixed at compile time in k_step; the bit
// kKinAlm selects the spherical-harmonic density observables instead of
// radial bins,
// kKinScf the self-consistent stellar potential
enum : int { kKinNone = 0, kKinV2 = 1, kKinGH4 = 2, kKinGHN = 3, kKinLOSVD = 4, kKinAlm = 8,
             kKinScf = 16 };

template <int KIN>
struct KinSlots {
    static constexpr int n = ((KIN & 7) == kKinGH4) ? 4 : ((KIN & 7) == kKinGHN) ? kMaxGH : 1;
};

// Non-zero kernels K_j of one phase-space point: the radial bin jr (K = 1),
// or with a_lm the mesh interval jr with the cloud-in-cell weight g of its
// inner radius and the direction (cos, sin of the polar angle; cos, sin of
// the azimuth); then kn kinematic entries j = jk + m with values k[m].
template <typename T, int KIN>
struct Kern {
    int jr, jk, kn;
    T k[KinSlots<KIN>::n];
    T g, ct, st, cp, sp;
};

// ------------------------------------------------------- spherical harmonics
// Real orthonormal harmonics Y_lm (Condon-Shortley phase) through the
// normalized associated Legendre functions Pn_l^m = N_lm P_l^m,
// N_lm = sqrt((2l + 1)/(4 pi) (l - m)!/(l + m)!):
//   Pn_0^0 = 1/sqrt(4 pi),  Pn_m^m = -sqrt((2m + 1)/(2m)) sin(t) Pn_{m-1}^{m-1},
//   Pn_{m+1}^m = sqrt(2m + 3) cos(t) Pn_m^m,
//   Pn_l^m = a_lm (cos(t) Pn_{l-1}^m - b_lm Pn_{l-2}^m),
//   a_lm = sqrt((4l^2 - 1)/(l^2 - m^2)),  b_lm = sqrt(((l-1)^2 - m^2)/(4(l-1)^2 - 1));
// Y_l0 = Pn_l^0, Y_l,m = sqrt2 Pn_l^m cos(m phi), Y_l,-m = sqrt2 Pn_l^m sin(m phi).
constexpr double csqrt(double x) {  // compile-time square root (Newton)
    double r = x > 1.0 ? x : 1.0;
    for (int i = 0; i < 64; ++i) r = 0.5 * (r + x / r);
    return r;
}

struct YlmCoef {
    double mm[kMaxLM + 1], m1[kMaxLM + 1], a[kMaxLM + 1][kMaxLM + 1], b[kMaxLM + 1][kMaxLM + 1];
    // theta derivatives: d Pn_l^m / dt = l cos(t) Qn_l^m - e_lm Qn_{l-1}^m with
    // Qn = Pn / sin(t) (m >= 1), e_lm = sqrt((2l + 1)(l^2 - m^2) / (2l - 1));
    // d Pn_l^0 / dt = sqrt(l (l + 1)) Pn_l^1 = s_l sin(t) Qn_l^1
    double e[kMaxLM + 1][kMaxLM + 1], s[kMaxLM + 1];
};

constexpr YlmCoef ylm_coef() {
    YlmCoef c{};
    for (int m = 0; m <= kMaxLM; ++m) {
        c.mm[m] = m > 0 ? csqrt((2.0 * m + 1.0) / (2.0 * m)) : 0.0;
        c.m1[m] = csqrt(2.0 * m + 3.0);
        for (int l = m + 2; l <= kMaxLM; ++l) {
            const double ll = double(l) * l, mm2 = double(m) * m, l1 = double(l - 1) * (l - 1);
            c.a[l][m] = csqrt((4.0 * ll - 1.0) / (ll - mm2));
            c.b[l][m] = csqrt((l1 - mm2) / (4.0 * l1 - 1.0));
        }
        for (int l = m + 1; l <= kMaxLM; ++l)
            c.e[l][m] = csqrt((2.0 * l + 1.0) * (double(l) * l - double(m) * m) / (2.0 * l - 1.0));
        c.s[m] = csqrt(double(m) * (m + 1.0));
    }
    return c;
}

__constant__ YlmCoef kYlm = ylm_coef();
constexpr YlmCoef kYlmC = ylm_coef();  // the same, folded where the indices are constant

// coefficient of the harmonics recurrences: from the folded copy when the
// degree is fixed at compile time (LMAX >= 0), else from constant memory
#define M2M_YC(LMAX, field) ((LMAX) >= 0 ? kYlmC.field : kYlm.field)

// f(l^2 + l + m, Y_lm) for every 0 <= l <= lmax, -l <= m <= l, at the
// direction (ct, st) = cos, sin of the polar angle and (cp, sp) of the azimuth
// LMAX >= 0: the degree is LMAX, fixed at compile time (loops unrolled,
// coefficients folded); LMAX < 0: the degree lmax
template <int LMAX, typename T, typename F>
__device__ __forceinline__ void ylm_walk_n(int lmax, T ct, T st, T cp, T sp, F&& f) {
    const int L = LMAX >= 0 ? LMAX : lmax;
    T pmm = T(0.282094791773878143);  // 1/sqrt(4 pi)
    T cm = T(1), sm = T(0);           // cos(m phi), sin(m phi)
#pragma unroll
    for (int m = 0; m <= (LMAX >= 0 ? LMAX : kMaxLM); ++m) {
        if (m > L) break;
        if (m > 0) {
            pmm = -T(M2M_YC(LMAX, mm[m])) * st * pmm;
            const T c = cm * cp - sm * sp;
            sm = sm * cp + cm * sp;
            cm = c;
        }
        const T c2 = T(1.41421356237309505) * cm, s2 = T(1.41421356237309505) * sm;
        auto emit = [&](int l, T pn) {
            if (m == 0) {
                f(l * l + l, pn);
            } else {
                f(l * l + l + m, pn * c2);
                f(l * l + l - m, pn * s2);
            }
        };
        emit(m, pmm);
        if (m < L) {
            T p2 = pmm, p1 = T(M2M_YC(LMAX, m1[m])) * ct * pmm;
            emit(m + 1, p1);
#pragma unroll
            for (int l = m + 2; l <= (LMAX >= 0 ? LMAX : kMaxLM); ++l) {
                if (l > L) break;
                const T p = T(M2M_YC(LMAX, a[l][m])) * (ct * p1 - T(M2M_YC(LMAX, b[l][m])) * p2);
                emit(l, p);
                p2 = p1;
                p1 = p;
            }
        }
    }
}

// the walk with the common degrees 2 and 4 unrolled
template <typename T, typename F>
__device__ __forceinline__ void ylm_walk(int lmax, T ct, T st, T cp, T sp, F&& f) {
    if (lmax == 4)
        ylm_walk_n<4>(4, ct, st, cp, sp, f);
    else if (lmax == 2)
        ylm_walk_n<2>(2, ct, st, cp, sp, f);
    else
        ylm_walk_n<-1>(lmax, ct, st, cp, sp, f);
}

template <typename T, typename A, int KIN>
__device__ __forceinline__ Kern<T, KIN> kernels(const Hot<T>& h, const Tabs<T, A>& tb, T x, T y,
                                                T z, T vz) {
    constexpr int KK = KIN & 7;
    Kern<T, KIN> o;
    const T R2 = x * x + y * y;
    const T r2 = R2 + z * z;
    o.jr = bin_of<T>(r2, tb.re2, h.n_r, (Mth<T>::log2_(r2) - h.lr0) * h.lrs, h.r2lo, h.r2hi);
    if ((KIN & kKinAlm) && o.jr >= 0) {
        // cloud-in-cell weight of the inner mesh radius (linear in r) and the
        // direction; r >= r_min > 0 here
        const T r = Mth<T>::sqrt_(r2);
        const T r0 = tb.rm[o.jr], r1 = tb.rm[o.jr + 1];
        o.g = (r1 - r) / (r1 - r0);
        const T ir = Mth<T>::rcp_(r);
        o.ct = z * ir;
        const T R = Mth<T>::sqrt_(R2);
        o.st = R * ir;
        const T iR = R > T(0) ? Mth<T>::rcp_(R) : T(0);
        o.cp = R > T(0) ? x * iR : T(1);
        o.sp = y * iR;
    }
    o.jk = -1;
    o.kn = 0;
    if (KK == kKinNone) return o;
    const int p = bin_of<T>(R2, tb.Re2, h.n_R, (Mth<T>::log2_(R2) - h.lR0) * h.lRs, h.R2lo, h.R2hi);
    if (p < 0) return o;
    const int base = h.jk0 + p * h.nk;
    if (KK == kKinV2) {
        o.jk = base;
        o.kn = 1;
        o.k[0] = vz * vz;
    } else if (KK == kKinGH4 || KK == kKinGHN) {
        // 2 sqrt(pi) u_n(nu) = sqrt2 e^{-nu^2/2} H_n(nu) / sqrt(2^n n!) by the
        // normalized three-term recurrence
        constexpr int NS = KinSlots<KIN>::n;
        const T nu = (vz - tb.Vp[p]) * tb.isp[p];
        const T g = T(1.41421356237309505) * Mth<T>::exp_(T(-0.5) * nu * nu);
        T hm = T(1);
        T hc = T(1.41421356237309505) * nu;
        o.jk = base;
        o.kn = (KK == kKinGH4) ? 4 : h.gh_nmax;
        o.k[0] = g * hc;
#pragma unroll
        for (int n = 1; n < NS; ++n) {
            if (KK == kKinGH4 || n < h.gh_nmax) {
                const T hn = T(kGhA[n]) * nu * hc - T(kGhB[n]) * hm;
                hm = hc;
                hc = hn;
                o.k[n] = g * hc;
            }
        }
    } else {
        const int b = bin_of<T>(vz, tb.ve, h.n_v, (vz - h.vmin) * h.vidv, h.vlo, h.vhi);
        if (b >= 0) {
            o.jk = base + b;
            o.kn = 1;
            o.k[0] = T(1);
        }
    }
    return o;
}

// ------------------------------------------------------------- potential ---
template <typename T>
__device__ __forceinline__ T phi_of(const Hot<T>& h, T r) {
    T p = -h.GMh / (r + h.a);
    if (h.GMn > T(0)) {
        const T q = r * h.irs;
        const T l = (q > T(1e-4)) ? Mth<T>::log1p_(q) / q : T(1) - q * (T(0.5) - q * T(1.0 / 3.0));
        p -= h.GMn * h.irs * l;
    }
    return p;
}

// the logarithmic halo v0^2/2 ln(r0^2 + R^2 + z^2/q^2) at R^2, z^2
template <typename T>
__device__ __forceinline__ T halo_phi(const Hot<T>& h, T R2, T z2) {
    return T(0.5) * h.hv2 * Mth<T>::log_(h.hr02 + R2 + z2 * h.hiq2);
}

// s(r) with g = -s(r) * (x, y, z) for the spherical parts: G M(<r) / r^3
// (without the Hernquist stars for STARS = false)
template <typename T, bool STARS = true>
__device__ __forceinline__ T accel_of(const Hot<T>& h, T r) {
    if (!(r > T(0))) return T(0);
    const T ra = r + h.a;
    T s = STARS ? h.GMh * Mth<T>::rcp_(r * ra * ra) : T(0);
    if (h.GMn > T(0)) {
        const T q = r * h.irs;
        T m;
        if (q < T(Mth<T>::nfw_series_max)) {
            // ln(1+q) - q/(1+q) = sum_{k>=2} (-1)^k (k-1) q^k / k
            m = q * q *
                (T(0.5) -
                 q * (T(2.0 / 3.0) -
                      q * (T(0.75) - q * (T(0.8) - q * (T(5.0 / 6.0) - q * (T(6.0 / 7.0) - q * T(0.875)))))));
        } else {
            m = Mth<T>::log1p_(q) - q * Mth<T>::rcp_(T(1) + q);
        }
        s += h.GMn * m * Mth<T>::rcp_(r * r * r);
    }
    return s;
}

// Prior cell (k, l) -> k n_x + l of one phase-space point.
template <typename T>
__device__ __forceinline__ int cell_of(const Hot<T>& h, T x, T y, T z, T vx, T vy, T vz) {
    const T R2 = x * x + y * y;
    const T r = Mth<T>::sqrt_(R2 + z * z);
    T E = T(0.5) * (vx * vx + vy * vy + vz * vz) + phi_of<T>(h, r);
    if (h.halo) E += halo_phi<T>(h, R2, z * z);
    const T lx = y * vz - z * vy, ly = z * vx - x * vz, lz = x * vy - y * vx;
    const T L = Mth<T>::sqrt_(lx * lx + ly * ly + lz * lz);
    T xc;
    if (!h.halo && !(E < T(0))) {
        xc = T(0);  // unbound: no circular orbit
    } else if (!(E > h.phi0)) {
        xc = T(1);
    } else {
        // radius of the circular orbit of energy E (in the equatorial plane)
        // from the table of ln r_c(ln zeta), zeta = (E - Phi(0)) / (-E), or
        // (E - Phi(0)) / v0^2 with the logarithmic halo; in FP64 refined by
        // Newton steps on E_c(r) = Phi(r) + r Phi'(r) / 2 = E
        const T zeta = h.halo ? (E - h.phi0) * h.iv2 : (E - h.phi0) / (-E);
        const T t = (Mth<T>::log_(zeta) - h.lz0) * h.ilz;
        const T tc = fmin(fmax(t, T(0)), T(kLcTable - 2));
        const int i = (int)tc;
        const T f = t - T(i);  // extrapolates linearly beyond the table
        T rc = Mth<T>::exp_(h.lctab[i] + f * (h.lctab[i + 1] - h.lctab[i]));
        if (sizeof(T) == 8) {
            for (int it = 0; it < 2; ++it) {
                T s = accel_of<T>(h, rc);
                T Ec = phi_of<T>(h, rc);
                const T ra = rc + h.a;
                T dEc = T(0.5) * s * rc + h.GMh * h.a / (ra * ra * ra);
                if (h.GMn > T(0)) {
                    const T q1 = T(1) + rc * h.irs;
                    dEc += T(0.5) * h.GMn * h.irs * h.irs / (q1 * q1);
                }
                if (h.halo) {
                    const T d = h.hr02 + rc * rc;
                    s += h.hv2 / d;
                    Ec += halo_phi<T>(h, rc * rc, T(0));
                    dEc += h.hv2 * rc * (T(2) * h.hr02 + rc * rc) / (d * d);
                }
                Ec += T(0.5) * s * rc * rc;
                const T rn = rc - (Ec - E) / dEc;
                rc = (rn > T(0)) ? rn : T(0.5) * rc;
            }
        }
        T sc = accel_of<T>(h, rc);
        if (h.halo) sc += h.hv2 * Mth<T>::rcp_(h.hr02 + rc * rc);
        const T Lc = rc * rc * Mth<T>::sqrt_(sc);  // r v_c, v_c^2 = r dPhi/dr
        xc = (Lc > T(0)) ? L / Lc : T(1);
    }
    // energy coordinate in bin units, linear in E or in exp(E); below E_lo
    // (or NaN) it clamps into bin 0
    const T ec = (h.cell_flags & 2) ? Mth<T>::exp_(E) : E;
    const T te = fmin((ec - h.E_lo) * h.E_scale, T(h.n_E));
    int k = (te >= T(0)) ? (int)te : 0;
    k = min(k, h.n_E - 1);
    const T tx = fmin(xc * T(h.n_x), T(h.n_x));
    int l = (tx >= T(0)) ? (int)tx : 0;
    l = min(l, h.n_x - 1);
    return k * h.n_x + l + (((h.cell_flags & 1) && lz < T(0)) ? h.cell_half : 0);
}

// ------------------------------------------------------------- accumulate --
// Add the kernels of one particle (weight w) into its private bin copies.
// FP64 bins: one FP64 LDS atomic add per kernel (gfx950 runs these about six
// times faster than FP32 LDS atomic adds). FP32 bins: every add returns the
// value it replaced, and the exact rounding error of the add (TwoSum) goes
// into the compensation array; all adds of the particle are issued before
// their errors are formed. The error terms are exact only if every value is
// rounded where the source rounds it: FP contraction is off in this part (a
// product fused into the error's add would differ from the value added).
__device__ __forceinline__ float two_sum_err(float old, float v) {
#pragma clang fp contract(off)
    const float t = old + v;  // the value the add stored
    const float bp = t - old;
    return (old - (t - bp)) + (v - bp);
}

// The a_lm part of a deposit of weight w: w g Y_lm at the inner mesh radius
// of the interval, w (1 - g) Y_lm at the outer one; add(j, value).
template <typename T, int KIN, typename Add>
__device__ __forceinline__ void deposit_alm(const Hot<T>& h, const Kern<T, KIN>& kk, T w,
                                            Add&& add) {
    const int b0 = kk.jr * h.nlm, b1 = b0 + h.nlm;
    const T wa = w * kk.g, wb = w * (T(1) - kk.g);
    ylm_walk(h.l_max, kk.ct, kk.st, kk.cp, kk.sp, [&](int lm, T Y) {
        add(b0 + lm, wa * Y);
        add(b1 + lm, wb * Y);
    });
}

template <typename T, int KIN>
__device__ __forceinline__ void deposit(const Hot<T>& h, const Tabs<T, float>& tb,
                                        const Kern<T, KIN>& kk, T u, int priv) {
#pragma clang fp contract(off)
    constexpr int NS = KinSlots<KIN>::n;
    const int kp = h.kp;
    const float wf = (float)(u * h.w0);
    float o_r = 0.f;
    float v[NS], o_k[NS];
#pragma unroll
    for (int m = 0; m < NS; ++m) v[m] = (float)(wf * kk.k[m]);
    if ((KIN & kKinAlm) && kk.jr >= 0)
        deposit_alm(h, kk, T(wf), [&](int j, T val) {
            const float vf = (float)val;
            const float o = atomicAdd(&tb.sum[j * kp + priv], vf);
            atomicAdd(&tb.comp[j * kp + priv], two_sum_err(o, vf));
        });
    if (!(KIN & kKinAlm) && kk.jr >= 0) o_r = atomicAdd(&tb.sum[kk.jr * kp + priv], wf);
#pragma unroll
    for (int m = 0; m < NS; ++m)
        if (m < kk.kn) o_k[m] = atomicAdd(&tb.sum[(kk.jk + m) * kp + priv], v[m]);
    if (!(KIN & kKinAlm) && kk.jr >= 0) atomicAdd(&tb.comp[kk.jr * kp + priv], two_sum_err(o_r, wf));
#pragma unroll
    for (int m = 0; m < NS; ++m)
        if (m < kk.kn) atomicAdd(&tb.comp[(kk.jk + m) * kp + priv], two_sum_err(o_k[m], v[m]));
}

template <typename T, int KIN>
__device__ __forceinline__ void deposit(const Hot<T>& h, const Tabs<T, double>& tb,
                                        const Kern<T, KIN>& kk, T u, int priv) {
    constexpr int NS = KinSlots<KIN>::n;
    const int kp = h.kp;
    const T w = u * h.w0;
    if ((KIN & kKinAlm) && kk.jr >= 0)
        deposit_alm(h, kk, w, [&](int j, T val) { atomicAdd(&tb.sum[j * kp + priv], (double)val); });
    if (!(KIN & kKinAlm) && kk.jr >= 0) atomicAdd(&tb.sum[kk.jr * kp + priv], (double)w);
#pragma unroll
    for (int m = 0; m < NS; ++m)
        if (m < kk.kn) atomicAdd(&tb.sum[(kk.jk + m) * kp + priv], (double)(w * kk.k[m]));
}


// ------------------------------------------------ self-consistent potential
// The stellar potential of the particles as a multipole expansion,
//   Phi_*(x) = sum_lm Phi_lm(r) Y_lm(theta, phi),
//   Phi_lm(r) = -4 pi G / (2l + 1) [r^-(l+1) A_lm(r) + r^l B_lm(r)],
//   A_lm(r) = sum_{r_i < r} m_i r_i^l Y_lm(x_i),  B_lm(r) = sum_{r_i >= r} m_i r_i^-(l+1) Y_lm(x_i),
// known at the nodes rho_k with the slope r dPhi_lm/dr (node table). The step
// kernel deposits u r^l Y_lm into the interval of each particle (0 below
// rho_0, k + 1 for rho_k <= r < rho_{k+1}, K beyond the last node) for
// intervals 0..K-1, and u r^-(l+1) Y_lm for intervals 1..K; the finalize
// forms the prefix and suffix sums at the nodes. Between nodes Phi_lm is the
// cubic Hermite interpolant in s = ln r; inside rho_0 the regular
// r^l (c0 + c1 r^2), beyond the last node the decaying c0 r^-(l+1) +
// c1 r^-(l+3), each with the value and slope of its end node. A particle
// with a non-finite radius deposits nothing.
template <typename T>
struct Scf {
    int K, L, nlm;
    T ls0, ih;       // ln rho_0, 1 / node spacing in ln r
    const T* rho;    // K node radii (LDS)
    // per interval q = 0..K and (l, m): (Phi, r dPhi/dr) at the inner and the
    // outer end node (LDS; the core and the outer interval repeat their one
    // node), one 4-vector per entry
    const T* tab;
    double* bins;    // 2 K nlm interval sums (LDS)
};

// LDS bytes of the expansion: sums, interval table and node radii
__host__ __device__ inline size_t scf_lds_bytes(int K, int L, size_t sz) {
    const size_t nlm = (size_t)(L + 1) * (size_t)(L + 1);
    return 8 * 2 * (size_t)K * nlm + sz * ((size_t)(K + 1) * nlm * 4 + (size_t)K) + 32;
}

template <typename T>
__device__ __forceinline__ int scf_interval(const Scf<T>& s, T r) {
    if (!(r >= s.rho[0])) return 0;
    if (r >= s.rho[s.K - 1]) return s.K;
    int k = (int)((Mth<T>::log_(r) - s.ls0) * s.ih);
    k = min(max(k, 0), s.K - 2);
    if (r < s.rho[k]) --k;  // the guess is within one interval
    else if (r >= s.rho[k + 1]) ++k;
    return k + 1;
}

// direction cosines of (x, y, z): cos, sin of the polar angle and of the
// azimuth (the +x azimuth on the z axis, the +z pole at the centre)
template <typename T>
__device__ __forceinline__ void scf_dir(T x, T y, T z, T r, T R, T& ct, T& st, T& cp, T& sp) {
    const T ir = r > T(0) ? Mth<T>::rcp_(r) : T(0);
    ct = r > T(0) ? z * ir : T(1);
    st = R * ir;
    const T iR = R > T(0) ? Mth<T>::rcp_(R) : T(0);
    cp = R > T(0) ? x * iR : T(1);
    sp = y * iR;
}

// deposit of one particle of weight u into the interval sums
template <typename T>
__device__ __forceinline__ void scf_deposit(const Scf<T>& s, T x, T y, T z, T u) {
    const T R2 = x * x + y * y;
    const T r = Mth<T>::sqrt_(R2 + z * z), R = Mth<T>::sqrt_(R2);
    T ct, st, cp, sp;
    scf_dir<T>(x, y, z, r, R, ct, st, cp, sp);
    if (!(r <= Mth<T>::max_)) return;  // inf or NaN
    const int q = scf_interval<T>(s, r);
    const T ir = r > T(0) ? Mth<T>::rcp_(r) : T(0);
    double* const A = q < s.K ? s.bins + q * s.nlm : nullptr;
    double* const B = q > 0 ? s.bins + (s.K + q - 1) * s.nlm : nullptr;
    T pmm = T(0.282094791773878143);  // 1/sqrt(4 pi)
    T cm = T(1), sm = T(0);
    T rm = u, irm = u * ir;  // u r^m, u r^-(m+1)
    for (int m = 0; m <= s.L; ++m) {
        if (m > 0) {
            pmm = -T(kYlm.mm[m]) * st * pmm;
            const T c = cm * cp - sm * sp;
            sm = sm * cp + cm * sp;
            cm = c;
            rm *= r;
            irm *= ir;
        }
        const T c2 = T(1.41421356237309505) * cm, s2 = T(1.41421356237309505) * sm;
        T p2 = T(0), p1 = pmm, rl = rm, irl = irm;
        for (int l = m; l <= s.L; ++l) {
            if (l == m + 1) {
                p2 = p1;
                p1 = T(kYlm.m1[m]) * ct * pmm;
            } else if (l > m + 1) {
                const T p = T(kYlm.a[l][m]) * (ct * p1 - T(kYlm.b[l][m]) * p2);
                p2 = p1;
                p1 = p;
            }
            if (l > m) {
                rl *= r;
                irl *= ir;
            }
            const int j = l * l + l;
            if (m == 0) {
                if (A) atomicAdd(&A[j], (double)(rl * p1));
                if (B) atomicAdd(&B[j], (double)(irl * p1));
            } else {
                const T yc = p1 * c2, ys = p1 * s2;
                if (A) {
                    atomicAdd(&A[j + m], (double)(rl * yc));
                    atomicAdd(&A[j - m], (double)(rl * ys));
                }
                if (B) {
                    atomicAdd(&B[j + m], (double)(irl * yc));
                    atomicAdd(&B[j - m], (double)(irl * ys));
                }
            }
        }
    }
}

// g = -grad Phi_* at (x, y, z): dPhi/dr, (1/r) dPhi/dtheta and
// (1/(r sin theta)) dPhi/dphi, with Qn = Pn / sin(theta) carried by the
// same recurrences as Pn (no division on the axis); zero at the centre.
// Phi_lm and r dPhi_lm/dr at r are linear in the four table values of the
// particle's interval: Hermite weights between nodes; in the core and
// beyond the last node the form u^n (P + (sg D - n P)(u^2 - 1)/2), u = v,
// n = l, sg = 1 inside rho_0 and u = 1/v, n = l + 1, sg = -1 beyond the last
// node (v = r over the end node), whose weights depend on l.
template <typename T, int VEC>
struct ScfQuad;
template <>
struct ScfQuad<float, 4> {
    using type = float4;
};
template <>
struct ScfQuad<double, 4> {
    using type = double4;
};

// LMAX >= 0: the degree is LMAX, fixed at compile time (loops unrolled,
// coefficients folded); LMAX < 0: the fit's degree s.L
template <typename T, int LMAX>
__device__ __forceinline__ void scf_accel(const Scf<T>& s, T x, T y, T z, T& gx, T& gy, T& gz) {
    using Q4 = typename ScfQuad<T, 4>::type;
    const int L = LMAX >= 0 ? LMAX : s.L;
    gx = gy = gz = T(0);
    const T R2 = x * x + y * y, r2 = R2 + z * z;
    if (!(r2 > T(0))) return;
    const T r = Mth<T>::sqrt_(r2), R = Mth<T>::sqrt_(R2);
    T ct, st, cp, sp;
    scf_dir<T>(x, y, z, r, R, ct, st, cp, sp);
    const int nlm = s.nlm;
    const int q = scf_interval<T>(s, r);
    const bool outer = q == 0 || q == s.K;
    const Q4* const row = reinterpret_cast<const Q4*>(s.tab) + q * nlm;
    // interior: Hermite weights of (P0, D0, P1, D1) for the value (w) and the
    // slope (e); outer: u, sg, the offset of n over l, and the first power
    T w0 = T(0), w1 = T(0), w2 = T(0), w3 = T(0), e0 = T(0), e1 = T(0), e2 = T(0), e3 = T(0);
    T u = T(1), sg = T(1), dn = T(0), qh = T(0), u2 = T(1), pw0 = T(1);
    if (!outer) {
        const T t = fmin(fmax((Mth<T>::log_(r) - s.ls0) * s.ih - T(q - 1), T(0)), T(1));
        const T t2 = t * t, t3 = t2 * t, h = Mth<T>::rcp_(s.ih);
        w0 = T(2) * t3 - T(3) * t2 + T(1);
        w1 = h * (t3 - T(2) * t2 + t);
        w2 = T(3) * t2 - T(2) * t3;
        w3 = h * (t3 - t2);
        e0 = (T(6) * t2 - T(6) * t) * s.ih;
        e1 = T(3) * t2 - T(4) * t + T(1);
        e2 = -e0;
        e3 = T(3) * t2 - T(2) * t;
    } else {
        const T v = r * Mth<T>::rcp_(s.rho[q == 0 ? 0 : s.K - 1]);
        u = q == 0 ? v : Mth<T>::rcp_(v);
        sg = q == 0 ? T(1) : T(-1);
        dn = q == 0 ? T(0) : T(1);
        pw0 = q == 0 ? T(1) : u;
        u2 = u * u;
        qh = T(0.5) * (u2 - T(1));
    }
    // Phi_lm (f) and r dPhi_lm/dr (d) of entry lm, degree l, pw = u^n
    auto radial = [&](int l, int lm, T pw, T& f, T& d) {
        const Q4 t = row[lm];
        const T n = T(l) + dn;
        const T g = n * qh + u2;
        const T W0 = outer ? pw * (T(1) - n * qh) : w0;
        const T W1 = outer ? pw * sg * qh : w1;
        const T E0 = outer ? sg * pw * n * (T(1) - g) : e0;
        const T E1 = outer ? pw * g : e1;
        f = W0 * t.x + W1 * t.y + w2 * t.z + w3 * t.w;
        d = E0 * t.x + E1 * t.y + e2 * t.z + e3 * t.w;
    };
    T fr = T(0), fth = T(0), fph = T(0);
    T pmm = T(0.282094791773878143);  // Pn_m^m (m = 0: 1/sqrt(4 pi))
    T cm = T(1), sm = T(0), pwm = pw0;
#pragma unroll
    for (int m = 0; m <= (LMAX >= 0 ? LMAX : kMaxLM); ++m) {
        if (m > L) break;
        T qmm = T(0);  // Qn_m^m
        if (m > 0) {
            qmm = -T(M2M_YC(LMAX, mm[m])) * pmm;
            pmm = st * qmm;
            const T c = cm * cp - sm * sp;
            sm = sm * cp + cm * sp;
            cm = c;
            pwm *= u;
        }
        const T c2 = T(1.41421356237309505) * cm, s2 = T(1.41421356237309505) * sm;
        // column m: X_l = Pn_l^0 for m = 0, Qn_l^m for m >= 1; along the m = 0
        // column also Y_l = Qn_l^1, for d Pn_l^0 / dtheta = s_l sin(theta) Qn_l^1
        T x2 = T(0), x1 = (m == 0) ? pmm : qmm, pw = pwm;
        T y2 = T(0), y1 = T(0);
#pragma unroll
        for (int l = m; l <= (LMAX >= 0 ? LMAX : kMaxLM); ++l) {
            if (l > L) break;
            if (l == m + 1) {
                x2 = x1;
                x1 = T(M2M_YC(LMAX, m1[m])) * ct * x1;
            } else if (l > m + 1) {
                const T xn = T(M2M_YC(LMAX, a[l][m])) * (ct * x1 - T(M2M_YC(LMAX, b[l][m])) * x2);
                x2 = x1;
                x1 = xn;
            }
            if (l > m) pw *= u;
            const int j = l * l + l;
            if (m == 0) {
                if (l == 1) {
                    y1 = -T(M2M_YC(LMAX, mm[1])) * T(0.282094791773878143);
                } else if (l == 2) {
                    y2 = y1;
                    y1 = T(M2M_YC(LMAX, m1[1])) * ct * y1;
                } else if (l > 2) {
                    const T yn = T(M2M_YC(LMAX, a[l][1])) * (ct * y1 - T(M2M_YC(LMAX, b[l][1])) * y2);
                    y2 = y1;
                    y1 = yn;
                }
                T f, d;
                radial(l, j, pw, f, d);
                fr += d * x1;
                fth += f * T(M2M_YC(LMAX, s[l])) * st * y1;
            } else {
                const T pn = st * x1;
                const T dth = T(l) * ct * x1 - (l > m ? T(M2M_YC(LMAX, e[l][m])) * x2 : T(0));
                T fp, dp, fm, dm;
                radial(l, j + m, pw, fp, dp);
                radial(l, j - m, pw, fm, dm);
                fr += (dp * c2 + dm * s2) * pn;
                fth += (fp * c2 + fm * s2) * dth;
                fph += T(m) * x1 * (fm * c2 - fp * s2);
            }
        }
    }
    const T ir = Mth<T>::rcp_(r);
    const T gr = fr * ir, gt = fth * ir, gp = fph * ir;
    gx = -(gr * st * cp + gt * ct * cp - gp * sp);
    gy = -(gr * st * sp + gt * ct * sp + gp * cp);
    gz = -(gr * ct - gt * st);
}

}  // namespace
}  // namespace m2m

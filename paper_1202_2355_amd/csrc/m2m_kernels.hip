// HIP kernels (gfx950) of the chi^2 M2M step with moving priors.
//
// One M2M step is two kernels:
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
    __device__ static float log1p_(float x) { return log1pf(x); }
    __device__ static float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
    static constexpr float nfw_series_max = 0.1f;
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
    T E_lo, E_scale, lz0, ilz;
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
    h.E_lo = T(fd.E_lo);
    h.E_scale = T(fd.E_scale);
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
// radial bins
enum : int { kKinNone = 0, kKinV2 = 1, kKinGH4 = 2, kKinGHN = 3, kKinLOSVD = 4, kKinAlm = 8 };

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
    }
    return c;
}

__constant__ YlmCoef kYlm = ylm_coef();

// f(l^2 + l + m, Y_lm) for every 0 <= l <= lmax, -l <= m <= l, at the
// direction (ct, st) = cos, sin of the polar angle and (cp, sp) of the azimuth
template <typename T, typename F>
__device__ __forceinline__ void ylm_walk(int lmax, T ct, T st, T cp, T sp, F&& f) {
    T pmm = T(0.282094791773878143);  // 1/sqrt(4 pi)
    T cm = T(1), sm = T(0);           // cos(m phi), sin(m phi)
    for (int m = 0; m <= lmax; ++m) {
        if (m > 0) {
            pmm = -T(kYlm.mm[m]) * st * pmm;
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
        if (m < lmax) {
            T p2 = pmm, p1 = T(kYlm.m1[m]) * ct * pmm;
            emit(m + 1, p1);
            for (int l = m + 2; l <= lmax; ++l) {
                const T p = T(kYlm.a[l][m]) * (ct * p1 - T(kYlm.b[l][m]) * p2);
                emit(l, p);
                p2 = p1;
                p1 = p;
            }
        }
    }
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

// s(r) with g = -s(r) * (x, y, z): G M(<r) / r^3
template <typename T>
__device__ __forceinline__ T accel_of(const Hot<T>& h, T r) {
    if (!(r > T(0))) return T(0);
    const T ra = r + h.a;
    T s = h.GMh * Mth<T>::rcp_(r * ra * ra);
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
    const T r = Mth<T>::sqrt_(x * x + y * y + z * z);
    const T E = T(0.5) * (vx * vx + vy * vy + vz * vz) + phi_of<T>(h, r);
    const T lx = y * vz - z * vy, ly = z * vx - x * vz, lz = x * vy - y * vx;
    const T L = Mth<T>::sqrt_(lx * lx + ly * ly + lz * lz);
    T xc;
    if (!(E < T(0))) {
        xc = T(0);
    } else if (!(E > h.phi0)) {
        xc = T(1);
    } else {
        // radius of the circular orbit of energy E from the table of
        // ln r_c(ln zeta), zeta = (E - Phi(0)) / (-E); in FP64 refined by
        // Newton steps on E_c(r) = Phi(r) + r Phi'(r) / 2 = E
        const T zeta = (E - h.phi0) / (-E);
        const T t = (Mth<T>::log_(zeta) - h.lz0) * h.ilz;
        const T tc = fmin(fmax(t, T(0)), T(kLcTable - 2));
        const int i = (int)tc;
        const T f = t - T(i);  // extrapolates linearly beyond the table
        T rc = Mth<T>::exp_(h.lctab[i] + f * (h.lctab[i + 1] - h.lctab[i]));
        if (sizeof(T) == 8) {
            for (int it = 0; it < 2; ++it) {
                const T s = accel_of<T>(h, rc);
                const T Ec = phi_of<T>(h, rc) + T(0.5) * s * rc * rc;
                const T ra = rc + h.a;
                T dEc = T(0.5) * s * rc + h.GMh * h.a / (ra * ra * ra);
                if (h.GMn > T(0)) {
                    const T q1 = T(1) + rc * h.irs;
                    dEc += T(0.5) * h.GMn * h.irs * h.irs / (q1 * q1);
                }
                const T rn = rc - (Ec - E) / dEc;
                rc = (rn > T(0)) ? rn : T(0.5) * rc;
            }
        }
        const T Lc = rc * rc * Mth<T>::sqrt_(accel_of<T>(h, rc));  // sqrt(G M(<r) r)
        xc = (Lc > T(0)) ? L / Lc : T(1);
    }
    const T te = fmin((E - h.E_lo) * h.E_scale, T(h.n_E));
    int k = (te >= T(0)) ? (int)te : 0;
    k = min(k, h.n_E - 1);
    const T tx = fmin(xc * T(h.n_x), T(h.n_x));
    int l = (tx >= T(0)) ? (int)tx : 0;
    l = min(l, h.n_x - 1);
    return k * h.n_x + l;
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
    bool step, cells_mode, observe, init, correct, refresh;
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

__device__ __forceinline__ Flags flags_of(const FitDev& fd, const Snap& ss, int32_t mode) {
    Flags f;
    f.step = (mode & kModeStep) != 0;
    f.cells_mode = (mode & kModeCells) != 0;
    f.observe = (mode & kModeObserve) != 0;
    f.init = (mode & kModeInit) != 0;
    f.correct = f.step && ss.correct != 0;
    f.refresh = f.cells_mode || (f.correct && fd.entropy == 0 && fd.prior_every > 0 &&
                                 ((ss.kstep + 1) % fd.prior_every) == 0);
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

// Thin-plate smoothing of the prior grid with the GCV-chosen lambda (Sec.
// 2.3.2, eq. smooth_grid) by the block that ends a refresh step. On the grid
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
__device__ void smooth_priors(const FitDev& fd, double* sa, double* sb, double* tE, double* tX,
                              double* buf, int* sidx, double* smean) {
    static_assert(2 * kSmoothMaxPoints <= kFinWaves * kFinCols, "GCV scores and lambdas in buf");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nE = fd.n_E, nx = fd.n_x, n = nE * nx;
    const G<const double> w0 = gmem<const double>(fd.cdata);
    const G<double> gp = gmem(fd.gprior);
    const G<T> uc = gmem<T>(fd.ucell);
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
        const double hE = (fd.E_hi - fd.E_lo) / nE, hx = 1.0 / nx;
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

template <typename T>
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
    const bool bins = jb.kind == 0;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int col = jb.col0 + lane;
    const bool in = col < (bins ? fd.J : fd.C);

    // observable columns: the rows and the smoothing inputs are requested
    // before the fit's state is known (their latency overlaps its load)
    double acc = 0.0, acc2 = 0.0;
    double yt0 = 0.0, sg = 1.0, Yj = 0.0;
    if (bins && !cells_mode && in) {
        group_sum<16>(fd, true, col, jb.n_tiles, wave, acc, acc2);
        if (wave == 0 && !observe) {
            yt0 = gmem(fd.ytil)[col];
            sg = gmem(fd.sigma)[col];
            Yj = gmem(fd.Y)[col];
        }
    }
    const Snap ss = snap_of(gst);
    if (step && ss.steps_left <= 0) return;  // uniform: the fit is idle
    const Flags f = flags_of(fd, ss, mode);
    if (bins && cells_mode) return;
    if (!bins && !f.refresh) return;
    // cell columns, read only on refresh steps
    if (!bins && in) group_sum<8>(fd, false, col, jb.n_tiles, wave, acc, acc2);
    part[wave][lane] = acc;
    part2[wave][lane] = acc2;
    __syncthreads();
    if (wave == 0) {
        double tot = 0.0, tot2 = 0.0;
        for (int w = 0; w < kFinWaves; ++w) {
            tot += part[w][lane];
            tot2 += part2[w][lane];
        }
        (void)column_epilogue<T>(fd, bins, jb.col0, f, tot, tot2, yt0, sg, Yj, lane);
    }
    // the last job of this fit ends the step; in observe mode the same
    // hand-over runs on a separate counter and changes no state
    const uint32_t n_part = (cells_mode ? 0u : (uint32_t)fd.n_bin_jobs) +
                            (f.refresh ? (uint32_t)fd.n_cell_jobs : 0u);
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
        smooth_priors<T>(fd, sgrid[0], sgrid[1], stab[0], stab[1], &part[0][0], &sidx, &smean);
    if (wave != 0) return;
    const double chi2 =
        cells_mode ? 0.0 : chi2_of_parts(static_cast<const double*>(fd.chi2_part), fd.n_bin_jobs, lane);
    if (lane != 0) return;
    *ticket = 0u;
    if (observe) return;
    end_step(fd, gst, f, ss, chi2);
}

// the jobs of the fits of a table (batches)
template <typename T>
__global__ __launch_bounds__(kFinThreads) void k_finalize(const FitDev* __restrict__ fits,
                                                         const FinJob* __restrict__ jobs,
                                                         int32_t mode) {
    const FinJob jb = jobs[blockIdx.x];
    finalize_job<T>(fits[jb.fit], jb, mode);
}

// one fit, its description passed by value: block b < n_bin_jobs takes bin
// columns, the others cell columns, over n_rows tile rows
template <typename T>
__global__ __launch_bounds__(kFinThreads) void k_finalize1(const FitDev fd, int32_t n_rows,
                                                          int32_t mode) {
    const int b = blockIdx.x;
    const bool bins = b < fd.n_bin_jobs;
    const FinJob jb{0, bins ? 0 : 1, (bins ? b : b - fd.n_bin_jobs) * kFinCols, n_rows};
    finalize_job<T>(fd, jb, mode);
}

// ------------------------------------------------------------- step --------
// A particle store that writes through L2 (agent-scope relaxed atomic store):
// the value reaches the memory-side cache at once instead of staying dirty in
// L2 until the write-back at the end of the kernel.
template <typename T>
__device__ __forceinline__ void put_wt(G<T> p, T v) {
    __hip_atomic_store((T*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T, typename A, int BLOCK, int KIN>
__device__ __forceinline__ void step_tile(const FitDev& fd, const Tile& tl, int32_t mode) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const bool step = (mode & kModeStep) != 0;

    // particle arrays from the tile start (32-bit offsets within the tile);
    // the first particle of every lane is requested before anything else so
    // that its latency overlaps the set-up below
    const G<T> __restrict__ X = gmem<T>(fd.x) + tl.begin;
    const G<T> __restrict__ Y = gmem<T>(fd.y) + tl.begin;
    const G<T> __restrict__ Z = gmem<T>(fd.z) + tl.begin;
    const G<T> __restrict__ VX = gmem<T>(fd.vx) + tl.begin;
    const G<T> __restrict__ VY = gmem<T>(fd.vy) + tl.begin;
    const G<T> __restrict__ VZ = gmem<T>(fd.vz) + tl.begin;
    const G<T> __restrict__ U = gmem<T>(fd.u) + tl.begin;
    const G<T> __restrict__ UH = gmem<T>(fd.uh) + tl.begin;
    const G<uint16_t> __restrict__ CI = gmem(fd.cidx) + tl.begin;
    const int len = (int)(tl.end - tl.begin);
    int i = threadIdx.x;
    T nx = T(0), ny = T(0), nz = T(0), nvx = T(0), nvy = T(0), nvz = T(0), nu = T(0), nh = T(1);
    if (i < len) {
        nx = X[i];
        ny = Y[i];
        nz = Z[i];
        nvx = VX[i];
        nvy = VY[i];
        nvz = VZ[i];
        nu = U[i];
        if (step) nh = UH[i];
    }

    const G<const FitState> st = gmem<const FitState>(fd.st);
    if (step && st->steps_left <= 0) return;  // uniform: the fit is idle
    const bool cells_only = (mode & kModeCells) != 0;
    const bool correct = step && st->correct != 0;
    const bool refresh = cells_only || (correct && fd.entropy == 0 && fd.prior_every > 0 &&
                                        ((st->kstep + 1) % fd.prior_every) == 0);
    const bool assign = step && st->assign_pending != 0;
    const bool deposit_on = !cells_only;
    const bool push = step;
    const bool wt = (mode & kModeWriteThrough) != 0;
    const Hot<T> h = hot_of<T>(fd);
    const int J = h.J, C = h.C, kp = h.kp;

    Tabs<T, A> tb = carve<T, A>(lds_raw, J, kp, h.n_r, h.n_R, h.n_v, C);
    const int priv = threadIdx.x & (kp - 1);
    {
        const G<const T> rp = gmem<const T>(fd.rp);
        for (int j = threadIdx.x; j < J; j += BLOCK) tb.rp[j] = rp[j];
        for (int j = threadIdx.x; j < J * kp; j += BLOCK) {
            tb.sum[j] = A(0);
            if (sizeof(A) == 4) tb.comp[j] = A(0);
        }
        if (refresh)
            for (int j = threadIdx.x; j < C; j += BLOCK) {
                tb.csum[j] = 0.0;
                tb.ccnt[j] = 0u;
            }
        const G<const T> re2 = gmem<const T>(fd.redge2);
        for (int j = threadIdx.x; j <= h.n_r; j += BLOCK) tb.re2[j] = re2[j];
        if (KIN & kKinAlm) {
            const G<const T> rm = gmem<const T>(fd.rmesh);
            for (int j = threadIdx.x; j <= h.n_r; j += BLOCK) tb.rm[j] = rm[j];
        }
        const G<const T> Re2 = gmem<const T>(fd.Redge2);
        for (int j = threadIdx.x; j <= h.n_R; j += BLOCK) tb.Re2[j] = Re2[j];
        const G<const T> ve = gmem<const T>(fd.vedge);
        for (int j = threadIdx.x; j <= h.n_v; j += BLOCK) tb.ve[j] = ve[j];
        const G<const T> Vp = gmem<const T>(fd.Vp);
        const G<const T> isp = gmem<const T>(fd.isp);
        for (int j = threadIdx.x; j < h.n_R; j += BLOCK) {
            tb.Vp[j] = Vp[j];
            tb.isp[j] = isp[j];
        }
    }
    const G<double> row = gmem(fd.partials) + (size_t)tl.row * (size_t)fd.row_len;
    const G<const T> __restrict__ ucell = gmem<const T>(fd.ucell);
    const bool need_uh = correct || assign;
    __syncthreads();

    // software pipeline: the loads of the next particle are in flight while
    // the current one is computed
    for (; i < len; i += BLOCK) {
        T x = nx, y = ny, z = nz, vx = nvx, vy = nvy, vz = nvz, u = nu, uh = nh;
        const int inext = i + BLOCK;
        if (inext < len) {
            nx = X[inext];
            ny = Y[inext];
            nz = Z[inext];
            nvx = VX[inext];
            nvy = VY[inext];
            nvz = VZ[inext];
            nu = U[inext];
            if (need_uh) nh = UH[inext];
        }
        // the prior of the particle's cell at the last refresh (same
        // phase-space point: no push in between)
        if (assign) uh = ucell[min((int)CI[i], C - 1)];
        if (correct) {
            // force of change at z^k with the residuals of step k
            const Kern<T, KIN> kk = kernels<T, A, KIN>(h, tb, x, y, z, vz);
            T chi = T(0);
            if ((KIN & kKinAlm) && kk.jr >= 0) {
                const int b0 = kk.jr * h.nlm, b1 = b0 + h.nlm;
                const T g1 = T(1) - kk.g;
                ylm_walk(h.l_max, kk.ct, kk.st, kk.cp, kk.sp, [&](int lm, T Y) {
                    chi += Y * (kk.g * tb.rp[b0 + lm] + g1 * tb.rp[b1 + lm]);
                });
            } else if (kk.jr >= 0) {
                chi = tb.rp[kk.jr];
            }
#pragma unroll
            for (int m = 0; m < KinSlots<KIN>::n; ++m)
                if (m < kk.kn) chi += kk.k[m] * tb.rp[kk.jk + m];
            const T lr = Mth<T>::log_(u * Mth<T>::rcp_(uh));
            u = u * Mth<T>::exp_(-h.foc_mu * (lr + h.foc_cs) - chi);
        }
        if (push) {
            x += h.hdt * vx;
            y += h.hdt * vy;
            z += h.hdt * vz;
            const T s = accel_of<T>(h, Mth<T>::sqrt_(x * x + y * y + z * z)) * h.dt;
            vx -= s * x;
            vy -= s * y;
            vz -= s * z;
            x += h.hdt * vx;
            y += h.hdt * vy;
            z += h.hdt * vz;
        }
        if (deposit_on) deposit<T, KIN>(h, tb, kernels<T, A, KIN>(h, tb, x, y, z, vz), u, priv);
        if (refresh) {
            const int c = cell_of<T>(h, x, y, z, vx, vy, vz);
            atomicAdd(&tb.csum[c], (double)u);
            atomicAdd(&tb.ccnt[c], 1u);
            CI[i] = (uint16_t)c;
        }
        if (push && wt) {
            put_wt(X + i, x);
            put_wt(Y + i, y);
            put_wt(Z + i, z);
            put_wt(VX + i, vx);
            put_wt(VY + i, vy);
            put_wt(VZ + i, vz);
            if (correct) put_wt(U + i, u);
            if (assign) put_wt(UH + i, uh);
        } else if (push) {
            X[i] = x;
            Y[i] = y;
            Z[i] = z;
            VX[i] = vx;
            VY[i] = vy;
            VZ[i] = vz;
            if (correct) U[i] = u;
            if (assign) UH[i] = uh;
        }
    }
    __syncthreads();
    if (deposit_on)
        for (int j = threadIdx.x; j < J; j += BLOCK) {
            double t = 0.0;
            for (int g = 0; g < kp; ++g) {
                t += (double)tb.sum[j * kp + g];
                if (sizeof(A) == 4) t += (double)tb.comp[j * kp + g];
            }
            row[j] = t;
        }
    if (refresh)
        for (int j = threadIdx.x; j < C; j += BLOCK) {
            row[J + j] = tb.csum[j];
            row[J + C + j] = (double)tb.ccnt[j];
        }
}

// the tiles of the fits of a table (batches)
template <typename T, typename A, int BLOCK, int KIN>
__global__ __launch_bounds__(BLOCK) void k_step(const FitDev* __restrict__ fits,
                                                const Tile* __restrict__ tiles, int32_t mode) {
    const Tile tl = tiles[blockIdx.x];
    step_tile<T, A, BLOCK, KIN>(fits[tl.fit], tl, mode);
}

// one fit, its description passed by value; block t takes tile t of the
// fit split into gridDim.x tiles
template <typename T, typename A, int BLOCK, int KIN>
__global__ __launch_bounds__(BLOCK) void k_step1(const FitDev fd, int32_t mode) {
    step_tile<T, A, BLOCK, KIN>(fd, tile_of(fd.n, (int)blockIdx.x, (int)gridDim.x, 0, 0), mode);
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
template <typename T, typename A, int BLOCK, int KIN>
hipError_t launch_step_t(const FitDev* fits, const Tile* tiles, const FitDev* one, int n_tiles,
                         size_t lds, int32_t mode, hipStream_t s) {
    if (one)
        hipLaunchKernelGGL((k_step1<T, A, BLOCK, KIN>), dim3(n_tiles), dim3(BLOCK), lds, s, *one,
                           mode);
    else
        hipLaunchKernelGGL((k_step<T, A, BLOCK, KIN>), dim3(n_tiles), dim3(BLOCK), lds, s, fits,
                           tiles, mode);
    return hipGetLastError();
}

template <typename T, typename A, int BLOCK>
hipError_t launch_step_kin(int kin, const FitDev* fits, const Tile* tiles, const FitDev* one,
                           int n_tiles, size_t lds, int32_t mode, hipStream_t s) {
    switch (kin) {
        case kKinNone: return launch_step_t<T, A, BLOCK, kKinNone>(fits, tiles, one, n_tiles, lds, mode, s);
        case kKinV2: return launch_step_t<T, A, BLOCK, kKinV2>(fits, tiles, one, n_tiles, lds, mode, s);
        case kKinGH4: return launch_step_t<T, A, BLOCK, kKinGH4>(fits, tiles, one, n_tiles, lds, mode, s);
        case kKinGHN: return launch_step_t<T, A, BLOCK, kKinGHN>(fits, tiles, one, n_tiles, lds, mode, s);
        case kKinLOSVD: return launch_step_t<T, A, BLOCK, kKinLOSVD>(fits, tiles, one, n_tiles, lds, mode, s);
        case kKinAlm | kKinNone: return launch_step_t<T, A, BLOCK, kKinAlm | kKinNone>(fits, tiles, one, n_tiles, lds, mode, s);
        case kKinAlm | kKinV2: return launch_step_t<T, A, BLOCK, kKinAlm | kKinV2>(fits, tiles, one, n_tiles, lds, mode, s);
        case kKinAlm | kKinGH4: return launch_step_t<T, A, BLOCK, kKinAlm | kKinGH4>(fits, tiles, one, n_tiles, lds, mode, s);
        case kKinAlm | kKinGHN: return launch_step_t<T, A, BLOCK, kKinAlm | kKinGHN>(fits, tiles, one, n_tiles, lds, mode, s);
        case kKinAlm | kKinLOSVD: return launch_step_t<T, A, BLOCK, kKinAlm | kKinLOSVD>(fits, tiles, one, n_tiles, lds, mode, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_step_any(bool f64, bool acc64, int block, int kin, const FitDev* fits,
                           const Tile* tiles, const FitDev* one, int n_tiles, size_t lds,
                           int32_t mode, hipStream_t s) {
    if (n_tiles <= 0) return hipSuccess;
    if (f64) return launch_step_kin<double, double, 256>(kin, fits, tiles, one, n_tiles, lds, mode, s);
    if (acc64) {
        if (block == 256) return launch_step_kin<float, double, 256>(kin, fits, tiles, one, n_tiles, lds, mode, s);
        if (block == 512) return launch_step_kin<float, double, 512>(kin, fits, tiles, one, n_tiles, lds, mode, s);
        if (block == 1024) return launch_step_kin<float, double, 1024>(kin, fits, tiles, one, n_tiles, lds, mode, s);
    } else {
        if (block == 256) return launch_step_kin<float, float, 256>(kin, fits, tiles, one, n_tiles, lds, mode, s);
        if (block == 512) return launch_step_kin<float, float, 512>(kin, fits, tiles, one, n_tiles, lds, mode, s);
        if (block == 1024) return launch_step_kin<float, float, 1024>(kin, fits, tiles, one, n_tiles, lds, mode, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

size_t step_lds_bytes(bool f64, bool acc64, int J, int n_r, int n_R, int n_v, int kpriv, int C) {
    (void)acc64;  // FP64 sums and FP32 sum + compensation both take 8 bytes per bin copy
    const size_t sz = f64 ? 8 : 4;
    const size_t bins = (size_t)J * (size_t)kpriv * 8 + (size_t)C * 8 + (size_t)((C + 1) & ~1) * 4;
    const size_t tabs = ((size_t)J + 2 * (size_t)(n_r + 1) + (size_t)(n_R + 1) + (size_t)(n_v + 1) +
                         2 * (size_t)n_R) * sz;
    return ((bins + tabs + 15) / 16) * 16;
}

// Private bin copies: as many as fit in 48 KiB of LDS, at most 8.
int private_copies(bool f64, int J) {
    (void)f64;
    const size_t per = (size_t)J * 8;
    int k = 8;
    while (k > 1 && per * (size_t)k > 48 * 1024) k >>= 1;
    return k;
}

int kin_class(int kin, int gh_nmax, int dens) {
    const int alm = dens == 1 ? kKinAlm : 0;
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
                           int n_jobs, int32_t mode, hipStream_t s) {
    if (n_jobs <= 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL(k_finalize<double>, dim3(n_jobs), dim3(kFinThreads), 0, s, fits, jobs,
                           mode);
    else
        hipLaunchKernelGGL(k_finalize<float>, dim3(n_jobs), dim3(kFinThreads), 0, s, fits, jobs,
                           mode);
    (void)n_fits;
    return hipGetLastError();
}

hipError_t launch_finalize1(bool f64, const FitDev& fd, int n_rows, int32_t mode, hipStream_t s) {
    const int n_jobs = fd.n_bin_jobs + fd.n_cell_jobs;
    if (n_jobs <= 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL(k_finalize1<double>, dim3(n_jobs), dim3(kFinThreads), 0, s, fd, n_rows,
                           mode);
    else
        hipLaunchKernelGGL(k_finalize1<float>, dim3(n_jobs), dim3(kFinThreads), 0, s, fd, n_rows,
                           mode);
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

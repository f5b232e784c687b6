// The fused step kernel (k_step for batches, k_step1 for one fit) and its
// compile-time dispatch; each step unit (m2m_step_*.hip) instantiates it for
// one particle-state / accumulator type pair.
#pragma once

#include "m2m_device.h"

namespace m2m {
namespace {

// ------------------------------------------------------------- step --------
// A particle store that writes through L2 (agent-scope relaxed atomic store):
// the value reaches the memory-side cache at once instead of staying dirty in
// L2 until the write-back at the end of the kernel.
template <typename T>
__device__ __forceinline__ void put_wt(G<T> p, T v) {
    __hip_atomic_store((T*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// NT: nontemporal particle loads and stores (streamed states, kModeStream);
// a compile-time choice, as the compiler merges a load of the same address
// in both arms of a run-time branch and drops the hint. IL: the tiles take
// interleaved chunks (one fit, kModeInterleave), also a compile-time
// choice: as a run-time branch it slowed the contiguous loop of a
// cache-resident fit by 2-3 %.
template <typename T, typename A, int BLOCK, int KIN, bool NT = false, bool IL = false>
__device__ __forceinline__ void step_tile(const FitDev& fd, const Tile& tl, int32_t mode) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const bool step = (mode & kModeStep) != 0;

    // The tile's particles: its contiguous range (arrays from the tile start),
    // or (IL) the chunks of BLOCK consecutive particles t, t + n_rows,
    // t + 2 n_rows, ... of the fit for tile t of n_rows (arrays from the fit
    // start); 32-bit offsets either way. Interleaved, the blocks in flight
    // stream one narrow window of each array instead of a range each. The
    // first particle of every lane is requested before anything else so that
    // its latency overlaps the set-up below.
    constexpr bool il = IL;
    const int64_t off = il ? 0 : tl.begin;
    const G<T> __restrict__ X = gmem<T>(fd.x) + off;
    const G<T> __restrict__ Y = gmem<T>(fd.y) + off;
    const G<T> __restrict__ Z = gmem<T>(fd.z) + off;
    const G<T> __restrict__ VX = gmem<T>(fd.vx) + off;
    const G<T> __restrict__ VY = gmem<T>(fd.vy) + off;
    const G<T> __restrict__ VZ = gmem<T>(fd.vz) + off;
    const G<T> __restrict__ U = gmem<T>(fd.u) + off;
    const G<T> __restrict__ UH = gmem<T>(fd.uh) + off;
    const G<uint16_t> __restrict__ CI = gmem(fd.cidx) + off;
    const int len = (int)(il ? fd.n : tl.end - tl.begin);
    const int istep = il ? tl.n_rows * BLOCK : BLOCK;
    int i = il ? tl.row * BLOCK + (int)threadIdx.x : (int)threadIdx.x;
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
    const bool pot_only = (KIN & kKinScf) && (mode & kModePot) != 0;
    // the steps that rebuild the self-consistent potential deposit into its
    // interval sums after the push
    const bool scf_dep = (KIN & kKinScf) &&
                         (pot_only || (step && ((st->tstep + 1) % fd.scf_every) == 0));
    const bool correct = step && st->correct != 0;
    const bool refresh = cells_only || (correct && fd.entropy == 0 && fd.prior_every > 0 &&
                                        ((st->kstep + 1) % fd.prior_every) == 0);
    const bool assign = step && st->assign_pending != 0;
    const bool deposit_on = !cells_only && !pot_only;
    const bool push = step;
    const bool wt = (mode & kModeWriteThrough) != 0;
    constexpr bool nt = NT;
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
    // the self-consistent potential: the interval table (32-byte aligned),
    // interval sums and node radii after the tables; offsets from the LDS
    // base, so that the compiler keeps LDS loads and atomics
    Scf<T> sc{};
    if (KIN & kKinScf) {
        const int off = (int)(tb.end - lds_raw + 31) & ~31;
        sc.K = fd.scf_nr;
        sc.L = fd.scf_lmax;
        sc.nlm = (fd.scf_lmax + 1) * (fd.scf_lmax + 1);
        sc.ls0 = T(fd.scf_ls0);
        sc.ih = T(fd.scf_ih);
        const int K = sc.K, nlm = sc.nlm, ne = (K + 1) * nlm;
        T* tt = reinterpret_cast<T*>(lds_raw + off);
        double* sb = reinterpret_cast<double*>(tt + 4 * ne);
        T* rr = reinterpret_cast<T*>(sb + 2 * K * nlm);
        sc.tab = tt;
        sc.bins = sb;
        sc.rho = rr;
        if (push) {
            // interval q: (Phi, r dPhi/dr) at its inner and outer node; the
            // core (q = 0) and the outer interval (q = K) repeat their node
            const G<const double> stab = gmem<const double>(fd.scf_tab);
            for (int e = threadIdx.x; e < ne; e += BLOCK) {
                const int qq = e / nlm, lm = e - qq * nlm;
                const int ki = qq == 0 ? 0 : qq - 1, ko = qq == K ? K - 1 : qq;
                tt[4 * e] = T(stab[(ki * nlm + lm) * 2]);
                tt[4 * e + 1] = T(stab[(ki * nlm + lm) * 2 + 1]);
                tt[4 * e + 2] = T(stab[(ko * nlm + lm) * 2]);
                tt[4 * e + 3] = T(stab[(ko * nlm + lm) * 2 + 1]);
            }
        }
        const G<const double> srho = gmem<const double>(fd.scf_rho);
        for (int j = threadIdx.x; j < K; j += BLOCK) rr[j] = T(srho[j]);
        if (scf_dep)
            for (int j = threadIdx.x; j < 2 * K * nlm; j += BLOCK) sb[j] = 0.0;
    }
    const G<double> row = gmem(fd.partials) + (size_t)tl.row * (size_t)fd.row_len;
    const G<const T> __restrict__ ucell = gmem<const T>(fd.ucell);
    const bool need_uh = correct || assign;
    __syncthreads();

    // software pipeline: the loads of the next particle are in flight while
    // the current one is computed
    for (; i < len; i += istep) {
        T x = nx, y = ny, z = nz, vx = nvx, vy = nvy, vz = nvz, u = nu, uh = nh;
        const int inext = i + istep;
        if (inext < len) {
            if constexpr (nt) {
                nx = __builtin_nontemporal_load(X + inext);
                ny = __builtin_nontemporal_load(Y + inext);
                nz = __builtin_nontemporal_load(Z + inext);
                nvx = __builtin_nontemporal_load(VX + inext);
                nvy = __builtin_nontemporal_load(VY + inext);
                nvz = __builtin_nontemporal_load(VZ + inext);
                nu = __builtin_nontemporal_load(U + inext);
                if (need_uh) nh = __builtin_nontemporal_load(UH + inext);
            } else {
                nx = X[inext];
                ny = Y[inext];
                nz = Z[inext];
                nvx = VX[inext];
                nvy = VY[inext];
                nvz = VZ[inext];
                nu = U[inext];
                if (need_uh) nh = UH[inext];
            }
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
            const T R2 = x * x + y * y, z2 = z * z;
            // with the self-consistent potential the expansion takes the
            // place of the Hernquist stars
            T s = accel_of<T, (KIN & kKinScf) == 0>(h, Mth<T>::sqrt_(R2 + z2)) * h.dt;
            T sz = s;
            if (h.halo) {  // logarithmic halo: -v0^2 (x, y, z/q^2) / (r0^2 + R^2 + z^2/q^2)
                const T sh = h.hv2 * Mth<T>::rcp_(h.hr02 + R2 + z2 * h.hiq2) * h.dt;
                s += sh;
                sz += sh * h.hiq2;
            }
            vx -= s * x;
            vy -= s * y;
            vz -= sz * z;
            if (KIN & kKinScf) {
                T gx, gy, gz;
                // the common degrees with their loops unrolled
                if (sc.L == 4)
                    scf_accel<T, 4>(sc, x, y, z, gx, gy, gz);
                else if (sc.L == 2)
                    scf_accel<T, 2>(sc, x, y, z, gx, gy, gz);
                else
                    scf_accel<T, -1>(sc, x, y, z, gx, gy, gz);
                vx += h.dt * gx;
                vy += h.dt * gy;
                vz += h.dt * gz;
            }
            x += h.hdt * vx;
            y += h.hdt * vy;
            z += h.hdt * vz;
        }
        if (deposit_on) deposit<T, KIN>(h, tb, kernels<T, A, KIN>(h, tb, x, y, z, vz), u, priv);
        if ((KIN & kKinScf) && scf_dep) scf_deposit<T>(sc, x, y, z, u);
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
        } else if (nt && push) {
            __builtin_nontemporal_store(x, X + i);
            __builtin_nontemporal_store(y, Y + i);
            __builtin_nontemporal_store(z, Z + i);
            __builtin_nontemporal_store(vx, VX + i);
            __builtin_nontemporal_store(vy, VY + i);
            __builtin_nontemporal_store(vz, VZ + i);
            if (correct) __builtin_nontemporal_store(u, U + i);
            if (assign) __builtin_nontemporal_store(uh, UH + i);
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
    if ((KIN & kKinScf) && scf_dep)
        for (int j = threadIdx.x; j < fd.scf_P; j += BLOCK) row[fd.scf_col0 + j] = sc.bins[j];
}

// the tiles of the fits of a table (batches)
template <typename T, typename A, int BLOCK, int KIN, bool NT = false>
__global__ __launch_bounds__(BLOCK) void k_step(const FitDev* __restrict__ fits,
                                                const Tile* __restrict__ tiles, int32_t mode) {
    const Tile tl = tiles[blockIdx.x];
    step_tile<T, A, BLOCK, KIN, NT>(fits[tl.fit], tl, mode);
}

// The same for the kinds of observables whose step fits 64 VGPRs without
// spilling, compiled for 8 waves per SIMD, so that two blocks of 1024 threads
// share a CU and one block's set-up and tail overlap the other's streaming.
template <int KIN>
constexpr bool lean_kin() {
    return (KIN & (kKinAlm | kKinScf)) == 0 && (KIN & 7) != kKinGHN;
}

template <typename T, typename A, int BLOCK, int KIN, bool NT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(8))) void k_step_w8(
    const FitDev* __restrict__ fits, const Tile* __restrict__ tiles, int32_t mode) {
    const Tile tl = tiles[blockIdx.x];
    step_tile<T, A, BLOCK, KIN, NT>(fits[tl.fit], tl, mode);
}

// one fit, its description passed by value; block t takes tile t of the
// fit split into gridDim.x tiles
template <typename T, typename A, int BLOCK, int KIN, bool IL = false>
__global__ __launch_bounds__(BLOCK) void k_step1(const FitDev fd, int32_t mode) {
    step_tile<T, A, BLOCK, KIN, false, IL>(fd, tile_of(fd.n, (int)blockIdx.x, (int)gridDim.x, 0, 0),
                                           mode);
}


template <typename T, typename A, int BLOCK, int KIN>
hipError_t launch_step_t(const FitDev* fits, const Tile* tiles, const FitDev* one, int n_tiles,
                         size_t lds, int32_t mode, hipStream_t s) {
    if (one) {
        // interleaved tiles are built for the lean kinds with FP32 state and
        // FP64 bins; other fits keep contiguous ranges
        if constexpr (lean_kin<KIN>() && sizeof(T) == 4 && sizeof(A) == 8)
            if (mode & kModeInterleave) {
                hipLaunchKernelGGL((k_step1<T, A, BLOCK, KIN, true>), dim3(n_tiles), dim3(BLOCK), lds, s,
                                   *one, mode);
                return hipGetLastError();
            }
        hipLaunchKernelGGL((k_step1<T, A, BLOCK, KIN>), dim3(n_tiles), dim3(BLOCK), lds, s, *one,
                           mode);
    } else if constexpr (lean_kin<KIN>() && sizeof(T) == 4 && sizeof(A) == 8 && BLOCK == 1024) {
        if (mode & kModeStream)
            hipLaunchKernelGGL((k_step_w8<T, A, BLOCK, KIN, true>), dim3(n_tiles), dim3(BLOCK), lds, s,
                               fits, tiles, mode);
        else
            hipLaunchKernelGGL((k_step_w8<T, A, BLOCK, KIN, false>), dim3(n_tiles), dim3(BLOCK), lds, s,
                               fits, tiles, mode);
    } else if constexpr (lean_kin<KIN>() && sizeof(T) == 4 && sizeof(A) == 8) {
        if (mode & kModeStream)
            hipLaunchKernelGGL((k_step<T, A, BLOCK, KIN, true>), dim3(n_tiles), dim3(BLOCK), lds, s, fits,
                               tiles, mode);
        else
            hipLaunchKernelGGL((k_step<T, A, BLOCK, KIN, false>), dim3(n_tiles), dim3(BLOCK), lds, s, fits,
                               tiles, mode);
    }
    else
        hipLaunchKernelGGL((k_step<T, A, BLOCK, KIN>), dim3(n_tiles), dim3(BLOCK), lds, s, fits,
                           tiles, mode);
    return hipGetLastError();
}

// kinds of observables with the compile-time bits HI (a_lm, self-consistent
// potential) set
template <typename T, typename A, int BLOCK, int HI>
hipError_t launch_step_lo(int lo, const FitDev* fits, const Tile* tiles, const FitDev* one,
                          int n_tiles, size_t lds, int32_t mode, hipStream_t s) {
    switch (lo) {
        case kKinNone: return launch_step_t<T, A, BLOCK, HI | kKinNone>(fits, tiles, one, n_tiles, lds, mode, s);
        case kKinV2: return launch_step_t<T, A, BLOCK, HI | kKinV2>(fits, tiles, one, n_tiles, lds, mode, s);
        case kKinGH4: return launch_step_t<T, A, BLOCK, HI | kKinGH4>(fits, tiles, one, n_tiles, lds, mode, s);
        case kKinGHN: return launch_step_t<T, A, BLOCK, HI | kKinGHN>(fits, tiles, one, n_tiles, lds, mode, s);
        case kKinLOSVD: return launch_step_t<T, A, BLOCK, HI | kKinLOSVD>(fits, tiles, one, n_tiles, lds, mode, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, typename A, int BLOCK>
hipError_t launch_step_kin(int kin, const FitDev* fits, const Tile* tiles, const FitDev* one,
                           int n_tiles, size_t lds, int32_t mode, hipStream_t s) {
    const int lo = kin & 7;
    switch (kin & ~7) {
        case 0: return launch_step_lo<T, A, BLOCK, 0>(lo, fits, tiles, one, n_tiles, lds, mode, s);
        case kKinAlm: return launch_step_lo<T, A, BLOCK, kKinAlm>(lo, fits, tiles, one, n_tiles, lds, mode, s);
        case kKinScf: return launch_step_lo<T, A, BLOCK, kKinScf>(lo, fits, tiles, one, n_tiles, lds, mode, s);
        case kKinAlm | kKinScf:
            return launch_step_lo<T, A, BLOCK, kKinAlm | kKinScf>(lo, fits, tiles, one, n_tiles, lds, mode, s);
        default: return hipErrorInvalidValue;
    }
}


}  // namespace
}  // namespace m2m

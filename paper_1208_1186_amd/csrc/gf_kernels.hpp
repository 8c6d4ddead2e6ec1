// HIP kernels of the Fourier-accelerated steepest-descent iteration.
//
// One iteration (paper, Section 1 and Section 2.2):
//   k_fft_xy<fwd>  2D FFT over (x, y) planes of the four packed Delta fields
//   k_fft_zt       2D FFT over (z, t), multiply by (alpha/2) K(p)/V, inverse (z, t)
//   k_fft_xy<inv>  inverse 2D FFT over (x, y)  -> (alpha/2) Delta~
//   k_update       g = reunitarize(1 + (alpha/2) Delta~); U_mu(x) -> g(x) U_mu(x) g(x+mu)^dag
//   k_divergence   Delta of the new links, per-block FP64 sums of Re Tr U and Tr Delta Delta^dag
//   k_finalize     fixed-order FP64 sum of the block partials -> theta, F, stop flag
//
// Delta is traceless anti-Hermitian, so it is carried as four complex fields:
// Z0 = Delta01, Z1 = Delta02, Z2 = Delta12, Z3 = d0 + i d1 with Delta00 = i d0,
// Delta11 = i d1. The filter is linear with a real, even kernel, so filtering
// these four fields is the same as filtering the nine matrix elements.
#pragma once

#include "gf_device.hpp"
#include "gf_fft.hpp"

namespace gf {

constexpr int kSiteThreads = 256;

// ------------------------------------------------------------ layout kernels
// Canonical links (complex double [s][mu][3][3]) -> SoA planes. If reunit is
// set the matrix is first re-orthonormalised in double (used before rounding
// to float).
template <typename T, int NE>
__global__ void __launch_bounds__(kSiteThreads) k_pack(const double* __restrict__ canon, Links<T, NE> L,
                                                       int64_t vol, int reunit) {
    const int64_t s = (int64_t)blockIdx.x * kSiteThreads + threadIdx.x;
    if (s >= vol) return;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const double* src = canon + (s * 4 + mu) * 18;
        su3<double> u;
#pragma unroll
        for (int k = 0; k < 9; ++k) u.e[k / 3][k % 3] = {src[2 * k], src[2 * k + 1]};
        if (reunit) reunitarize(u);
        su3<T> v;
#pragma unroll
        for (int k = 0; k < 9; ++k) v.e[k / 3][k % 3] = {(T)u.e[k / 3][k % 3].re, (T)u.e[k / 3][k % 3].im};
        L.store(mu, s, v);
    }
}

// SoA planes -> canonical links; a two-row link gets its third row rebuilt in double.
template <typename T, int NE>
__global__ void __launch_bounds__(kSiteThreads) k_unpack(Links<T, NE> L, double* __restrict__ canon, int64_t vol) {
    const int64_t s = (int64_t)blockIdx.x * kSiteThreads + threadIdx.x;
    if (s >= vol) return;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        su3<double> u;
        const cx<T>* b = L.p + (size_t)(mu * NE) * L.ps + s;
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            cx<T> e = b[(size_t)k * L.ps];
            u.e[k / 3][k % 3] = {(double)e.re, (double)e.im};
        }
        if constexpr (NE == 6) third_row(u.e[0], u.e[1], u.e[2]);
        double* dst = canon + (s * 4 + mu) * 18;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            dst[2 * k] = u.e[k / 3][k % 3].re;
            dst[2 * k + 1] = u.e[k / 3][k % 3].im;
        }
    }
}

// Canonical matrix field (complex double [s][3][3]) -> four packed fields, times scale.
template <typename T>
__global__ void __launch_bounds__(kSiteThreads) k_field_pack(const double* __restrict__ f, cx<T>* __restrict__ Z,
                                                             size_t zps, int64_t vol, double scale) {
    const int64_t s = (int64_t)blockIdx.x * kSiteThreads + threadIdx.x;
    if (s >= vol) return;
    const double* m = f + s * 18;
    Z[s] = {(T)(m[2] * scale), (T)(m[3] * scale)};                 // (0,1)
    Z[zps + s] = {(T)(m[4] * scale), (T)(m[5] * scale)};           // (0,2)
    Z[2 * zps + s] = {(T)(m[10] * scale), (T)(m[11] * scale)};     // (1,2)
    Z[3 * zps + s] = {(T)(m[1] * scale), (T)(m[9] * scale)};       // Im(0,0), Im(1,1)
}

// Four packed fields -> canonical anti-Hermitian traceless matrix field.
template <typename T>
__global__ void __launch_bounds__(kSiteThreads) k_field_unpack(const cx<T>* __restrict__ Z, size_t zps,
                                                               double* __restrict__ f, int64_t vol) {
    const int64_t s = (int64_t)blockIdx.x * kSiteThreads + threadIdx.x;
    if (s >= vol) return;
    const cx<T> z0 = Z[s], z1 = Z[zps + s], z2 = Z[2 * zps + s], z3 = Z[3 * zps + s];
    double* m = f + s * 18;
    const double d0 = z3.re, d1 = z3.im;
    m[0] = 0.0;          m[1] = d0;
    m[2] = z0.re;        m[3] = z0.im;
    m[4] = z1.re;        m[5] = z1.im;
    m[6] = -(double)z0.re; m[7] = z0.im;
    m[8] = 0.0;          m[9] = d1;
    m[10] = z2.re;       m[11] = z2.im;
    m[12] = -(double)z1.re; m[13] = z1.im;
    m[14] = -(double)z2.re; m[15] = z2.im;
    m[16] = 0.0;         m[17] = -(d0 + d1);
}

// ------------------------------------------------------------- divergence
// Delta(x) from sum_mu [U_mu(x - mu) - U_mu(x)]; per-block FP64 partial sums
// of Re Tr U_mu(x) (for F) and of Tr Delta Delta^dag (for theta).
template <typename T, int NE>
__global__ void __launch_bounds__(kSiteThreads) k_divergence(Links<T, NE> L, cx<T>* __restrict__ Z, size_t zps,
                                                             Geom g, double2* __restrict__ part,
                                                             const Ctl* __restrict__ ctl, int force) {
    if (!force && ctl->done) return;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t s = (int64_t)b * kSiteThreads + threadIdx.x;
    double fsum = 0.0, tsum = 0.0;
    if (s < g.vol) {
        int c[4];
        site_coords(g, s, c);
        su3<T> m;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) m.e[i][j] = {T(0), T(0)};
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const su3<T> u = L.load(mu, s);
            const su3<T> ub = L.load(mu, site_back(g, s, c, mu));
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) m.e[i][j] = m.e[i][j] + (ub.e[i][j] - u.e[i][j]);
            fsum += (double)u.e[0][0].re + (double)u.e[1][1].re + (double)u.e[2][2].re;
        }
        const cx<T> z0 = m.e[0][1] - conj(m.e[1][0]);
        const cx<T> z1 = m.e[0][2] - conj(m.e[2][0]);
        const cx<T> z2 = m.e[1][2] - conj(m.e[2][1]);
        const T tr = (m.e[0][0].im + m.e[1][1].im + m.e[2][2].im) / T(3);
        const T d0 = T(2) * (m.e[0][0].im - tr), d1 = T(2) * (m.e[1][1].im - tr);
        Z[s] = z0;
        Z[zps + s] = z1;
        Z[2 * zps + s] = z2;
        Z[3 * zps + s] = {d0, d1};
        const double e0 = norm2(z0), e1 = norm2(z1), e2 = norm2(z2);
        const double dd0 = d0, dd1 = d1;
        tsum = 2.0 * (e0 + e1 + e2) + dd0 * dd0 + dd1 * dd1 + (dd0 + dd1) * (dd0 + dd1);
    }
    block_sum2<kSiteThreads>(fsum, tsum);
    if (threadIdx.x == 0) part[b] = make_double2(fsum, tsum);
}

// Fixed-order reduction of the block partials; sets theta, F and the stop flag.
__global__ void __launch_bounds__(256) k_finalize(const double2* __restrict__ part, int n, double inv3v,
                                                  double inv12v, Ctl* ctl, int force) {
    if (!force && ctl->done) return;
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        a += part[i].x;
        b += part[i].y;
    }
    block_sum2<256>(a, b);
    if (threadIdx.x == 0) {
        const double F = a * inv12v, th = b * inv3v;
        ctl->F = F;
        ctl->theta = th;
        const long long k = ctl->iters;
        ctl->hist_theta[k % kHist] = th;
        ctl->hist_F[k % kHist] = F;
        if (!isfinite(th)) {
            ctl->numeric = 1;
            ctl->done = 1;
        } else if (th < ctl->tol) {
            ctl->done = 1;
        }
    }
}

__global__ void k_set_tol(Ctl* ctl, double tol) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->tol = tol;
        ctl->done = (ctl->numeric || ctl->theta < tol) ? 1 : 0;
    }
}

// ------------------------------------------------------------------ update
template <typename T>
__device__ __forceinline__ su3<T> g_at(const cx<T>* __restrict__ Z, size_t zps, int64_t s) {
    return g_from_packed(Z[s], Z[zps + s], Z[2 * zps + s], Z[3 * zps + s]);
}

// U_mu(x) -> g(x) U_mu(x) g(x+mu)^dag, g = reunitarize(1 + Z(x)), Z holding
// (alpha/2) Delta~. Float links are re-orthonormalised on write; double
// links are stored as computed.
template <typename T, int NE>
__global__ void __launch_bounds__(kSiteThreads) k_update(Links<T, NE> L, const cx<T>* __restrict__ Z, size_t zps,
                                                         Geom g, Ctl* ctl, int count) {
    if (ctl->done) return;
    if (count && blockIdx.x == 0 && threadIdx.x == 0) ctl->iters = ctl->iters + 1;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t s = (int64_t)b * kSiteThreads + threadIdx.x;
    if (s >= g.vol) return;
    int c[4];
    site_coords(g, s, c);
    const su3<T> g0 = g_at(Z, zps, s);
    constexpr int NR = NE == 9 ? 3 : 2;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const su3<T> g1 = g_at(Z, zps, site_fwd(g, s, c, mu));
        const su3<T> u = L.load(mu, s);
        const su3<T> gu = mul_rows<T, NR>(g0, u);
        su3<T> un = mul_adj<T, NR>(gu, g1);
        if constexpr (sizeof(T) == 4) reunitarize(un);
        L.store(mu, s, un);
    }
}

// --------------------------------------------------------------------- FFT
// 2D FFT over the (x, y) plane. Each block takes G consecutive planes of one
// field (flattened plane index = field * Nz*Nt + z + Nz*t), stages them in LDS
// with rows padded to rs elements, transforms along x then y, writes back.
template <typename T, int EPT, bool INV>
__global__ void __launch_bounds__(1024) k_fft_xy(cx<T>* __restrict__ Z, size_t zps, int nx, int ny, int nzt, int G,
                                                 int rs, FftPlan px, FftPlan py, const cx<T>* __restrict__ twgx,
                                                 const cx<T>* __restrict__ twgy, const Ctl* __restrict__ ctl,
                                                 int force) {
    if (!force && ctl->done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T>* twx = reinterpret_cast<cx<T>*>(smem);
    cx<T>* twy = twx + nx;
    cx<T>* buf = twy + ny;
    const int nthr = blockDim.x;
    for (int i = threadIdx.x; i < nx; i += nthr) twx[i] = twgx[i];
    for (int i = threadIdx.x; i < ny; i += nthr) twy[i] = twgy[i];
    const int q0 = blockIdx.x * G;
    const int f = q0 / nzt, zt0 = q0 - f * nzt;
    cx<T>* gp = Z + (size_t)f * zps + (size_t)zt0 * nx * ny;
    const int E = G * nx * ny;
    for (int e = threadIdx.x; e < E; e += nthr) {
        const int row = e / nx, x = e - row * nx;
        buf[row * rs + x] = gp[e];
    }
    __syncthreads();
    fft_rows<EPT, T, INV>(buf, twx, px, 1, G * ny, G * ny, rs, 0);
    fft_rows<EPT, T, INV>(buf, twy, py, rs, G * nx, nx, 1, ny * rs);
    for (int e = threadIdx.x; e < E; e += nthr) {
        const int row = e / nx, x = e - row * nx;
        gp[e] = buf[row * rs + x];
    }
}

// 2D FFT over (z, t) for bx consecutive x columns at one y of one field,
// multiply every mode by coef / p^2(p) (coef = (alpha/2) p2max / V; zero mode
// -> 0; coef alone when no_fa), then the inverse (z, t) transform.
// LDS element (xo, z, t) sits at t*tsp + z*bx + xo.
template <typename T, int EPT>
__global__ void __launch_bounds__(1024) k_fft_zt(cx<T>* __restrict__ Z, size_t zps, int nx, int ny, int nz, int nt,
                                                 int bx, int tsp, FftPlan pz, FftPlan pt,
                                                 const cx<T>* __restrict__ twgz, const cx<T>* __restrict__ twgt,
                                                 const T* __restrict__ sin2, T coef, int no_fa,
                                                 const Ctl* __restrict__ ctl, int force) {
    if (!force && ctl->done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T>* twz = reinterpret_cast<cx<T>*>(smem);
    cx<T>* twt = twz + nz;
    cx<T>* buf = twt + nt;
    const int nthr = blockDim.x;
    for (int i = threadIdx.x; i < nz; i += nthr) twz[i] = twgz[i];
    for (int i = threadIdx.x; i < nt; i += nthr) twt[i] = twgt[i];
    const int nxb = nx / bx;
    const int xb = blockIdx.x % nxb;
    const int rest = blockIdx.x / nxb;
    const int y = rest % ny, f = rest / ny;
    const int x0 = xb * bx;
    cx<T>* gp = Z + (size_t)f * zps + x0 + (size_t)nx * y;
    const size_t pstep = (size_t)nx * ny;
    const int E = bx * nz * nt;
    for (int e = threadIdx.x; e < E; e += nthr) {
        const int xo = e % bx, zt = e / bx;
        const int z = zt % nz, t = zt / nz;
        buf[t * tsp + z * bx + xo] = gp[xo + zt * pstep];
    }
    __syncthreads();
    fft_rows<EPT, T, false>(buf, twz, pz, bx, nt * bx, bx, 1, tsp);
    fft_rows<EPT, T, false>(buf, twt, pt, tsp, nz * bx, nz * bx, 1, 0);
    const T* sx = sin2;
    const T* sy = sin2 + nx;
    const T* sz = sy + ny;
    const T* st = sz + nz;
    for (int e = threadIdx.x; e < E; e += nthr) {
        const int xo = e % bx, zt = e / bx;
        const int z = zt % nz, t = zt / nz;
        const T p2 = sx[x0 + xo] + sy[y] + sz[z] + st[t];
        const T mult = p2 > T(0) ? (no_fa ? coef : coef / p2) : T(0);
        const int li = t * tsp + z * bx + xo;
        buf[li] = cscale(buf[li], mult);
    }
    __syncthreads();
    fft_rows<EPT, T, true>(buf, twt, pt, tsp, nz * bx, nz * bx, 1, 0);
    fft_rows<EPT, T, true>(buf, twz, pz, bx, nt * bx, bx, 1, tsp);
    for (int e = threadIdx.x; e < E; e += nthr) {
        const int xo = e % bx, zt = e / bx;
        const int z = zt % nz, t = zt / nz;
        gp[xo + zt * pstep] = buf[t * tsp + z * bx + xo];
    }
}

}  // namespace gf

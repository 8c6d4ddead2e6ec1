// Temporal Wilson lines and their colour-singlet correlator, the quantity that
// the paper's Eq. (1) builds its singlet free energy from, on a gauge-fixed field:
//
//   W(x) = U_t(x, 0) U_t(x, 1) ... U_t(x, Nt-1)        (x a spatial site)
//   C(r) = 1/(3 Vs) sum_x Re Tr[W(x + r) W(x)^dagger]  (every spatial separation r)
//
// and C averaged over the shells of equal minimum-image r^2. The sum over x is
// a cyclic correlation of the nine matrix elements, done by FFT:
//   sum_x Tr[W(x + r) W(x)^dag] = (1/Vs) sum_p S(p) e^{+i p.r},  S(p) = sum_ab |W~_ab(p)|^2,
// with W~ the unnormalised forward transform over (x, y, z).
//
// Kernels, in launch order:
//   k_wilson_lines   the ordered products along t; each wave of a block takes a
//                    chunk of t for 64 consecutive spatial sites and wave 0
//                    multiplies the chunk products in order (HBM bound: every
//                    temporal link is read once)
//   k_wcorr_xy_fwd   forward (x, y) transform of one z plane of one element
//   k_wcorr_z        per column chunk: forward z transforms of the nine
//                    elements together, S summed over them, inverse z transform of S
//   k_wcorr_xy_inv   inverse (x, y) transform of S, Re * 1/(3 Vs^2) -> C(r)
//   k_wcorr_shells   one wave per shell: members summed in a fixed order
#pragma once

#include "gf_fft.hpp"

namespace gf {

constexpr int kWlSites = 64;  // spatial sites per k_wilson_lines block (one per lane)

// The temporal link of a site: at site*36 + 27 in canonical links ([site][mu][row][col], mu = 3), or
// at site*9 in a field of temporal links alone ([site][row][col]).
template <int STRIDE>
__device__ __forceinline__ su3<double> load_temporal(const double2* __restrict__ canon, size_t site) {
    const double2* p = canon + site * STRIDE + (STRIDE == 36 ? 27 : 0);
    su3<double> m;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double2 v = p[i * 3 + j];
            m.e[i][j] = {v.x, v.y};
        }
    return m;
}

// C chunks of nt / C consecutive t per spatial site; wave w of the block takes chunk w. STRIDE: 36
// for canonical links, 9 for a temporal-link field.
template <int C, int STRIDE>
__global__ void __launch_bounds__(64 * C) k_wilson_lines(const double2* __restrict__ canon, int vs, int nt,
                                                         cx<double>* __restrict__ W, size_t wps,
                                                         double2* __restrict__ lines) {
    __shared__ double part[(C > 1 ? C - 1 : 1) * 18 * kWlSites];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int xs = blockIdx.x * kWlSites + lane;
    const bool live = xs < vs;
    const int len = nt / C, t0 = w * len;
    su3<double> acc;
    if (live) {
        acc = load_temporal<STRIDE>(canon, (size_t)xs + (size_t)vs * t0);
        su3<double> nxt;
        if (len > 1) nxt = load_temporal<STRIDE>(canon, (size_t)xs + (size_t)vs * (t0 + 1));
        for (int t = t0 + 1; t < t0 + len; ++t) {
            const su3<double> cur = nxt;
            if (t + 1 < t0 + len) nxt = load_temporal<STRIDE>(canon, (size_t)xs + (size_t)vs * (t + 1));  // in flight
            acc = mul(acc, cur);
        }
    }
    if (C > 1) {
        if (w > 0 && live) {
            double* dst = part + (size_t)(w - 1) * 18 * kWlSites + lane;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                dst[(2 * k) * kWlSites] = acc.e[k / 3][k % 3].re;
                dst[(2 * k + 1) * kWlSites] = acc.e[k / 3][k % 3].im;
            }
        }
        __syncthreads();
        if (w != 0) return;
        if (live) {
            for (int c = 1; c < C; ++c) {  // in increasing t
                const double* src = part + (size_t)(c - 1) * 18 * kWlSites + lane;
                su3<double> p;
#pragma unroll
                for (int k = 0; k < 9; ++k) p.e[k / 3][k % 3] = {src[(2 * k) * kWlSites], src[(2 * k + 1) * kWlSites]};
                acc = mul(acc, p);
            }
        }
    }
    if (!live) return;
#pragma unroll
    for (int k = 0; k < 9; ++k) W[(size_t)k * wps + xs] = acc.e[k / 3][k % 3];
    if (lines) {
#pragma unroll
        for (int k = 0; k < 9; ++k) lines[(size_t)xs * 9 + k] = {acc.e[k / 3][k % 3].re, acc.e[k / 3][k % 3].im};
    }
}

// LDS: twiddles for x and y, then the plane with rows padded to rs elements.
template <int EPT>
__device__ __forceinline__ void wcorr_plane_fft(cx<double>* buf, const cx<double>* twx, const cx<double>* twy,
                                                const FftPlan& px, const FftPlan& py, int nx, int ny, int rs,
                                                bool inv) {
    if (inv) {
        fft_rows<EPT, double, true>(buf, twx, px, 1, ny, ny, rs, 0);
        fft_rows<EPT, double, true>(buf, twy, py, rs, nx, nx, 1, 0);
    } else {
        fft_rows<EPT, double, false>(buf, twx, px, 1, ny, ny, rs, 0);
        fft_rows<EPT, double, false>(buf, twy, py, rs, nx, nx, 1, 0);
    }
}

// Forward (x, y) transform in place: block (z, element).
template <int EPT>
__global__ void __launch_bounds__(1024) k_wcorr_xy_fwd(cx<double>* __restrict__ W, size_t wps, int nx, int ny,
                                                       int rs, FftPlan px, FftPlan py,
                                                       const cx<double>* __restrict__ twgx,
                                                       const cx<double>* __restrict__ twgy) {
    extern __shared__ __align__(16) unsigned char smem[];
    cx<double>* twx = reinterpret_cast<cx<double>*>(smem);
    cx<double>* twy = twx + nx;
    cx<double>* buf = twy + ny;
    const int nthr = blockDim.x;
    for (int i = threadIdx.x; i < nx; i += nthr) twx[i] = twgx[i];
    for (int i = threadIdx.x; i < ny; i += nthr) twy[i] = twgy[i];
    const int plane = nx * ny;
    cx<double>* g = W + (size_t)blockIdx.y * wps + (size_t)blockIdx.x * plane;
    for (int e = threadIdx.x; e < plane; e += nthr) {
        const int y = e / nx, x = e - y * nx;
        buf[y * rs + x] = g[e];
    }
    __syncthreads();
    wcorr_plane_fft<EPT>(buf, twx, twy, px, py, nx, ny, rs, false);
    for (int e = threadIdx.x; e < plane; e += nthr) {
        const int y = e / nx, x = e - y * nx;
        g[e] = buf[y * rs + x];
    }
}

// Block b takes the bx consecutive in-plane positions q0 = b*bx .. q0+bx-1 for every z and all nine
// elements at once (LDS element (f, b, z) at f*bx*nz + z*bx + b): forward z transforms of the 9*bx
// columns, S = sum_f |.|^2 in a fixed order, then the inverse z transform of S, written to Sg.
template <int EPT>
__global__ void __launch_bounds__(1024) k_wcorr_z(const cx<double>* __restrict__ W, size_t wps, int plane, int nz,
                                                  int bx, FftPlan pz, const cx<double>* __restrict__ twgz,
                                                  cx<double>* __restrict__ Sg) {
    extern __shared__ __align__(16) unsigned char smem[];
    cx<double>* twz = reinterpret_cast<cx<double>*>(smem);
    cx<double>* buf = twz + nz;
    const int E = bx * nz;
    cx<double>* sb = buf + 9 * E;
    const int nthr = blockDim.x;
    for (int i = threadIdx.x; i < nz; i += nthr) twz[i] = twgz[i];
    const int q0 = blockIdx.x * bx;
    for (int e = threadIdx.x; e < 9 * E; e += nthr) {
        const int f = e / E, r = e - f * E;
        const int z = r / bx, b = r - z * bx;
        buf[e] = W[(size_t)f * wps + (size_t)z * plane + q0 + b];
    }
    __syncthreads();
    fft_rows<EPT, double, false>(buf, twz, pz, bx, 9 * bx, bx, 1, E);
    for (int e = threadIdx.x; e < E; e += nthr) {
        double s = 0.0;
#pragma unroll
        for (int f = 0; f < 9; ++f) s += norm2(buf[f * E + e]);
        sb[e] = {s, 0.0};
    }
    __syncthreads();
    fft_rows<EPT, double, true>(sb, twz, pz, bx, bx, bx, 1, 0);
    for (int e = threadIdx.x; e < E; e += nthr) {
        const int z = e / bx, b = e - z * bx;
        Sg[(size_t)z * plane + q0 + b] = sb[e];
    }
}

// Inverse (x, y) transform of one z plane of S; C(r) = Re * scale, scale = 1/(3 Vs^2).
template <int EPT>
__global__ void __launch_bounds__(1024) k_wcorr_xy_inv(const cx<double>* __restrict__ Sg, int nx, int ny, int rs,
                                                       FftPlan px, FftPlan py, const cx<double>* __restrict__ twgx,
                                                       const cx<double>* __restrict__ twgy, double scale,
                                                       double* __restrict__ corr) {
    extern __shared__ __align__(16) unsigned char smem[];
    cx<double>* twx = reinterpret_cast<cx<double>*>(smem);
    cx<double>* twy = twx + nx;
    cx<double>* buf = twy + ny;
    const int nthr = blockDim.x;
    for (int i = threadIdx.x; i < nx; i += nthr) twx[i] = twgx[i];
    for (int i = threadIdx.x; i < ny; i += nthr) twy[i] = twgy[i];
    const int plane = nx * ny;
    const cx<double>* g = Sg + (size_t)blockIdx.x * plane;
    for (int e = threadIdx.x; e < plane; e += nthr) {
        const int y = e / nx, x = e - y * nx;
        buf[y * rs + x] = g[e];
    }
    __syncthreads();
    wcorr_plane_fft<EPT>(buf, twx, twy, px, py, nx, ny, rs, true);
    double* out = corr + (size_t)blockIdx.x * plane;
    for (int e = threadIdx.x; e < plane; e += nthr) {
        const int y = e / nx, x = e - y * nx;
        out[e] = buf[y * rs + x].re * scale;
    }
}

// Shell means: wave s sums corr over members[off[s] .. off[s+1]) lane-strided, then a fixed butterfly.
__global__ void __launch_bounds__(256) k_wcorr_shells(const double* __restrict__ corr, const int* __restrict__ off,
                                                      const int* __restrict__ members, int nshell,
                                                      double* __restrict__ out) {
    const int s = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (s >= nshell) return;
    const int a = off[s], b = off[s + 1];
    double v = 0.0;
    for (int i = a + lane; i < b; i += 64) v += corr[members[i]];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    if (lane == 0) out[s] = v / (double)(b - a);
}

}  // namespace gf

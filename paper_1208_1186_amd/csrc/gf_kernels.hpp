// HIP kernels of the Fourier-accelerated steepest-descent iteration.
//
// The links are kept implicitly: the input links U0 never change, and the
// gauge transform H accumulated by the updates is stored instead (rows 1-2,
// six planes), so that the current links are U_mu(x) = H(x) U0_mu(x)
// H(x+mu)^dag. One update U -> g U g(x+mu)^dag is then H -> g H: 96 bytes per
// site written instead of the 576 of four FP64 links (the iteration is
// memory-bound). One loop iteration, from k to k + 1 applied updates (paper,
// Section 1 for the method, Section 2.2 for the per-element FFT split 2D + 2D):
//   k_fft_xy<fwd>   Delta (buffer D) -> 2D FFT over (x, y) -> buffer Q; one more
//                   block, dispatched first, reduces the theta/F partials left by
//                   the loop kernel
//   k_fft_zt        in Q: 2D FFT over (z, t), times (alpha/2) K(p) / V, inverse
//   k_fft_xy_gauge  Q -> inverse 2D FFT over (x, y) -> g = reunitarize(1 +
//                   (alpha/2) Delta~), H_{k+1} = reunitarize(g H_k) -> the
//                   other transform buffer
//   k_update_measure  the links H U0 H(x+mu)^dag of H_{k+1}: their divergence
//                   -> D, FP64 block partials of F and theta
// The partials are reduced by the next iteration's k_fft_xy (or by k_finalize
// before the host reads the control block), in a fixed order.
//
// Delta is traceless anti-Hermitian, so it is carried as four complex fields:
// Z0 = Delta01, Z1 = Delta02, Z2 = Delta12, Z3 = d0 + i d1 with Delta00 = i d0,
// Delta11 = i d1. The filter is linear with a real, even kernel, so filtering
// these four fields is the same as filtering the nine matrix elements.
#pragma once

#include "gf_device.hpp"
#include "gf_fft.hpp"
#include "gf_learn.hpp"

namespace gf {

constexpr int kSiteThreads = 256;

// ------------------------------------------------------------ layout kernels
// The egress moves 64 sites per block through LDS: lane (site, mu) forms one link into LDS (mu is the
// wave's), and the block writes the sites' 64 x 576 contiguous bytes of canonical links with consecutive
// lanes on consecutive words. A site's row in LDS is 73 doubles (72 + 1), so that the 64 lanes of a wave
// writing their links do not meet on the same banks.
constexpr int kIoSites = 64;
constexpr int kIoRow = 73;

// Canonical links (complex double [s][mu][3][3]) -> the tiled input links, one site per thread (staging
// the records through LDS as the egress does measured slower here: 269 against 263 us in FP64, 403
// against 312 us in FP32 at 32^3 x 64). If reunit is set the matrix is first re-orthonormalised in
// double (used before rounding to float).
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

// Canonical matrix field (complex double [s][3][3]) -> four packed fields, times scale.
template <typename T>
__global__ void __launch_bounds__(kSiteThreads) k_field_pack(const double* __restrict__ f, cx<T>* __restrict__ Z,
                                                             size_t zps, int64_t vol, double scale) {
    const int64_t s = (int64_t)blockIdx.x * kSiteThreads + threadIdx.x;
    if (s >= vol) return;
    const double* m = f + s * 18;
    Z[s] = {(T)(m[2] * scale), (T)(m[3] * scale)};              // (0,1)
    Z[zps + s] = {(T)(m[4] * scale), (T)(m[5] * scale)};        // (0,2)
    Z[2 * zps + s] = {(T)(m[10] * scale), (T)(m[11] * scale)};  // (1,2)
    Z[3 * zps + s] = {(T)(m[1] * scale), (T)(m[9] * scale)};    // Im(0,0), Im(1,1)
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
    m[0] = 0.0;
    m[1] = d0;
    m[2] = z0.re;
    m[3] = z0.im;
    m[4] = z1.re;
    m[5] = z1.im;
    m[6] = -(double)z0.re;
    m[7] = z0.im;
    m[8] = 0.0;
    m[9] = d1;
    m[10] = z2.re;
    m[11] = z2.im;
    m[12] = -(double)z1.re;
    m[13] = z1.im;
    m[14] = -(double)z2.re;
    m[15] = z2.im;
    m[16] = 0.0;
    m[17] = -(d0 + d1);
}

// ------------------------------------------------------------ gauge field g
// g(x) and the transform H(x) are stored as their first two rows (six complex entries per site, in
// tiles of 64 sites); the third row follows from unitarity.
template <typename T>
__device__ __forceinline__ su3<T> g_rows_at(const cx<T>* __restrict__ G, int64_t s) {
    su3<T> g;
#pragma unroll
    for (int k = 0; k < 6; ++k) g.e[k / 3][k % 3] = G[tile_index(6, k, s)];
    third_row(g.e[0], g.e[1], g.e[2]);
    return g;
}

// Stored g rows -> canonical matrix field.
template <typename T>
__global__ void __launch_bounds__(kSiteThreads) k_gauge_unpack(const cx<T>* __restrict__ G, double* __restrict__ f,
                                                               int64_t vol) {
    const int64_t s = (int64_t)blockIdx.x * kSiteThreads + threadIdx.x;
    if (s >= vol) return;
    su3<double> g;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const cx<T> e = G[tile_index(6, k, s)];
        g.e[k / 3][k % 3] = {(double)e.re, (double)e.im};
    }
    third_row(g.e[0], g.e[1], g.e[2]);
    double* m = f + s * 18;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        m[2 * k] = g.e[k / 3][k % 3].re;
        m[2 * k + 1] = g.e[k / 3][k % 3].im;
    }
}

// Row 1-2 planes of a transform at site s, promoted to double, row 3 rebuilt in double.
template <typename T>
__device__ __forceinline__ su3<double> rows_at_fp64(const cx<T>* __restrict__ G, int64_t s) {
    su3<double> g;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const cx<T> e = G[tile_index(6, k, s)];
        g.e[k / 3][k % 3] = {(double)e.re, (double)e.im};
    }
    third_row(g.e[0], g.e[1], g.e[2]);
    return g;
}

// Egress: the current links U_mu(x) = H(x) U0_mu(x) H(x+mu)^dag -> canonical links (complex double
// [s][mu][3][3]), formed in double from the stored factors (float factors promoted exactly); with
// two-row storage rows 1-2 are formed and row 3 is rebuilt from them, as for the stored links. Lane
// (site, mu) forms one link; the block writes its 64 sites' links from LDS as one contiguous run.
template <typename T, int NE>
__global__ void __launch_bounds__(kSiteThreads) k_unpack_h(Links<T, NE> U0, const cx<T>* __restrict__ H, Geom g,
                                                           double* __restrict__ canon) {
    __shared__ double row[kIoSites * kIoRow];
    const int64_t s0 = (int64_t)blockIdx.x * kIoSites;
    const int nsite = (int)(g.vol - s0 < kIoSites ? g.vol - s0 : kIoSites);
    const int q = threadIdx.x & (kIoSites - 1);
    const int mu = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kIoSites);
    if (q < nsite) {
        const int64_t s = s0 + q;
        int c[4];
        site_coords(g, s, c);
        const su3<double> h0 = rows_at_fp64(H, s);
        su3<double> u;
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            const cx<T> e = U0.p[U0.at(mu, k, s)];
            u.e[k / 3][k % 3] = {(double)e.re, (double)e.im};
        }
        if constexpr (NE == 6) third_row(u.e[0], u.e[1], u.e[2]);
        const su3<double> h1 = rows_at_fp64(H, site_fwd(g, s, c, mu));
        su3<double> v;
        if constexpr (NE == 6) {  // two-row storage: the third row of the result is rebuilt from its first two
            v = mul_adj<double, 2>(mul_rows<double, 2>(h0, u), h1);
            third_row(v.e[0], v.e[1], v.e[2]);
        } else {
            v = mul_adj<double, 3>(mul(h0, u), h1);
        }
        double* m = row + q * kIoRow + mu * 18;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            m[2 * k] = v.e[k / 3][k % 3].re;
            m[2 * k + 1] = v.e[k / 3][k % 3].im;
        }
    }
    __syncthreads();
    double* dst = canon + s0 * 72;
    for (int i = threadIdx.x; i < nsite * 72; i += kSiteThreads) dst[i] = row[(i / 72) * kIoRow + i % 72];
}

// ------------------------------------------------------------ reductions
// Fixed-order FP64 sum of n block partials (F part, theta part) by the
// calling block, independent of its size: 256 virtual lanes each add every
// 256th partial in increasing order, then a fixed pairwise tree. Thread 0
// publishes theta, F, the history entry and the stop flag; with advance set
// it first counts one more applied update.
__device__ __forceinline__ void reduce_partials(const double2* __restrict__ part, int n, double inv3v,
                                                double inv12v, Ctl* ctl, int advance) {
    __shared__ double ra[256], rb[256];
    for (int vt = threadIdx.x; vt < 256; vt += blockDim.x) {
        double a = 0.0, b = 0.0;
        for (int i0 = vt; i0 < n; i0 += 16 * 256) {
            double2 p[16];  // 16 loads in flight: the chain waits on memory latency, not on the adds
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                const int i = i0 + k * 256;
                p[k] = i < n ? part[i] : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int k = 0; k < 16; ++k) {
                a += p[k].x;
                b += p[k].y;
            }
        }
        ra[vt] = a;
        rb[vt] = b;
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        for (int vt = threadIdx.x; vt < h; vt += blockDim.x) {
            ra[vt] += ra[vt + h];
            rb[vt] += rb[vt + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double F = ra[0] * inv12v, th = rb[0] * inv3v;
        const long long k = ctl->iters + (advance ? 1 : 0);
        const bool worse = advance && ctl->guard && (!isfinite(th) || th > ctl->theta || F < ctl->F - 1e-14);
        ctl->iters = k;
        ctl->pending = 0;
        ctl->F = F;
        ctl->theta = th;
        ctl->hist_theta[k % kHist] = th;
        ctl->hist_F[k % kHist] = F;
        if (worse) {
            ctl->rejected = 1;
            ctl->done = 1;
        } else if (!isfinite(th)) {
            ctl->numeric = 1;
            ctl->done = 1;
        } else if (th < ctl->tol) {
            ctl->done = 1;
        }
    }
}

// mode 0: reduce a standalone measurement of the current links;
// mode 1: reduce the loop kernel's partials if they are still pending.
__global__ void __launch_bounds__(256) k_finalize(const double2* __restrict__ part, int n, double inv3v,
                                                  double inv12v, Ctl* ctl, int mode, Batch bt) {
    const size_t bo = boff(bt);
    part = bshift(part, bo);
    ctl = bshift(ctl, bo);
    if (mode == 1 && !ctl->pending) return;
    reduce_partials(part, n, inv3v, inv12v, ctl, mode);
}

// Current link U_mu(y) = H(y) U0_mu(y) H(y+mu)^dag (all three rows), yf the site y + mu.
template <typename T, int NE>
__device__ __forceinline__ su3<T> link_h(const Links<T, NE>& U0, const cx<T>* __restrict__ H, int mu, int64_t y,
                                         int64_t yf) {
    const su3<T> u = U0.load(mu, y);
    return mul_adj<T, 3>(mul(g_rows_at(H, y), u), g_rows_at(H, yf));
}

// y + d for a direction d known only at run time (a switch, so that no array is indexed by d).
__device__ __forceinline__ int64_t fwd_site(const Geom& g, int64_t y, const int cy[4], int d) {
    switch (d) {
        case 0: return site_fwd(g, y, cy, 0);
        case 1: return site_fwd(g, y, cy, 1);
        case 2: return site_fwd(g, y, cy, 2);
        default: return site_fwd(g, y, cy, 3);
    }
}

// Plaquette of the current links (gauge invariant, for checks): per site the six (mu < nu) loops
// Re Tr[U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag] = Re sum_ij A_ij conj(B_ij)
// with A = U_mu(x) U_nu(x+mu), B = U_nu(x) U_mu(x+nu), every link formed from H and U0; one FP64
// partial per block.
template <typename T, int NE>
__global__ void __launch_bounds__(kSiteThreads) k_plaquette_h(Links<T, NE> U0, const cx<T>* __restrict__ H, Geom g,
                                                              double2* __restrict__ part) {
    const int64_t s = (int64_t)blockIdx.x * kSiteThreads + threadIdx.x;
    double sum = 0.0, none = 0.0;
    if (s < g.vol) {
        int c[4];
        site_coords(g, s, c);
#pragma unroll 1
        for (int mu = 0; mu < 4; ++mu) {
            const int64_t sm = fwd_site(g, s, c, mu);
            int cm[4];
            site_coords(g, sm, cm);
            const su3<T> um = link_h(U0, H, mu, s, sm);
#pragma unroll 1
            for (int nu = mu + 1; nu < 4; ++nu) {
                const int64_t sn = fwd_site(g, s, c, nu);
                int cn[4];
                site_coords(g, sn, cn);
                const su3<T> a = mul(um, link_h(U0, H, nu, sm, fwd_site(g, sm, cm, nu)));
                const su3<T> b = mul(link_h(U0, H, nu, s, sn), link_h(U0, H, mu, sn, fwd_site(g, sn, cn, mu)));
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    const cx<T> x = a.e[k / 3][k % 3], y = b.e[k / 3][k % 3];
                    sum += (double)x.re * y.re + (double)x.im * y.im;
                }
            }
        }
    }
    block_sum2<kSiteThreads>(sum, none);
    if (threadIdx.x == 0) part[blockIdx.x] = make_double2(sum, 0.0);
}

// Fixed-order sum of n block partials (.x) times scale into ctl->plaquette (one block of 256).
__global__ void __launch_bounds__(256) k_plaquette_sum(const double2* __restrict__ part, int n, double scale,
                                                       Ctl* ctl) {
    __shared__ double r[256];
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) a += part[i].x;
    r[threadIdx.x] = a;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) r[threadIdx.x] += r[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) ctl->plaquette = r[0] * scale;
}

// Copy the leading words of n control blocks (cs bytes apart) into a dense array.
__global__ void __launch_bounds__(64) k_gather_heads(const unsigned char* __restrict__ ctl0, size_t cs, int words,
                                                     unsigned long long* __restrict__ out) {
    const unsigned long long* src = reinterpret_cast<const unsigned long long*>(ctl0 + (size_t)blockIdx.x * cs);
    for (int i = threadIdx.x; i < words; i += 64) out[(size_t)blockIdx.x * words + i] = src[i];
}

// Forget a rejected update: the count goes back to k (the links of step k are
// still in their buffer; the caller re-measures them).
__global__ void k_rollback(Ctl* ctl, long long k) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->iters = k;
        ctl->done = 0;
        ctl->pending = 0;
        ctl->rejected = 0;
    }
}

__global__ void k_set_guard(Ctl* ctl, int on) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->guard = on;
        ctl->rejected = 0;
    }
}

__global__ void k_set_tol(Ctl* ctl, double tol) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctl->tol = tol;
        ctl->done = (ctl->numeric || ctl->theta < tol) ? 1 : 0;
    }
}

// ------------------------------------------------------- single update
template <typename T>
__device__ __forceinline__ su3<T> g_at_packed(const cx<T>* __restrict__ Z, size_t zps, int64_t s, bool exact) {
    return g_from_packed(Z[s], Z[zps + s], Z[2 * zps + s], Z[3 * zps + s], exact);
}

// H <- reunitarize(g H): rows 1-2 of g times H (third row rebuilt), Gram-Schmidt (in double for float).
template <typename T>
__device__ __forceinline__ su3<T> gauge_times(const su3<T>& g, su3<T> h) {
    third_row(h.e[0], h.e[1], h.e[2]);
    su3<T> r = mul_rows<T, 2>(g, h);
    reunitarize_fp64(r);
    return r;
}

// One update of the stored transform in place, H(x) <- reunitarize(g(x) H(x)), g = reunitarize(1 + Z(x))
// with Z holding (alpha/2) Delta~ packed: the current links become g U g(x+mu)^dag. Used by the
// single-stage entry point (the loop does the same in the inverse (x, y) pass).
template <typename T>
__global__ void __launch_bounds__(kSiteThreads) k_h_update(const cx<T>* __restrict__ Z, size_t zps, cx<T>* __restrict__ H,
                                                           int64_t vol, int exact) {
    const int64_t s = (int64_t)blockIdx.x * kSiteThreads + threadIdx.x;
    if (s >= vol) return;
    su3<T> h;
#pragma unroll
    for (int k = 0; k < 6; ++k) h.e[k / 3][k % 3] = H[tile_index(6, k, s)];
    const su3<T> r = gauge_times(g_at_packed(Z, zps, s, exact != 0), h);
#pragma unroll
    for (int k = 0; k < 6; ++k) H[tile_index(6, k, s)] = r.e[k / 3][k % 3];
}

// ------------------------------------------------ loop kernel: update + divergence
// Anti-Hermitian part of a 3x3 matrix, kept as the nine reals that Delta needs:
// X01 - conj(X10), X02 - conj(X20), X12 - conj(X21) and Im X00, Im X11, Im X22.
template <typename T>
struct AhAcc {
    cx<T> o01, o02, o12;
    T d0, d1, d2;
    __device__ __forceinline__ void zero() {
        o01 = o02 = o12 = {T(0), T(0)};
        d0 = d1 = d2 = T(0);
    }
    __device__ __forceinline__ void set(const su3<T>& x) {
        o01 = x.e[0][1] - conj(x.e[1][0]);
        o02 = x.e[0][2] - conj(x.e[2][0]);
        o12 = x.e[1][2] - conj(x.e[2][1]);
        d0 = x.e[0][0].im;
        d1 = x.e[1][1].im;
        d2 = x.e[2][2].im;
    }
    __device__ __forceinline__ void sub(const AhAcc& b) {
        o01 = o01 - b.o01;
        o02 = o02 - b.o02;
        o12 = o12 - b.o12;
        d0 -= b.d0;
        d1 -= b.d1;
        d2 -= b.d2;
    }
};

// Sum over the four lanes l, l^16, l^32, l^48 of a wave (all four receive the
// same bits): two cross-row swaps on gfx950 (v_permlane16_swap /
// v_permlane32_swap), each followed by an add of the swapped pair.
__device__ __forceinline__ float xor_sum4(float v) {
    auto a = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    v = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    auto b = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(b[0]) + __uint_as_float(b[1]);
}
__device__ __forceinline__ double xor_sum4(double v) {
    unsigned lo = __double2loint(v), hi = __double2hiint(v);
    auto al = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    auto ah = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    v = __hiloint2double(ah[0], al[0]) + __hiloint2double(ah[1], al[1]);
    lo = __double2loint(v);
    hi = __double2hiint(v);
    auto bl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    auto bh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return __hiloint2double(bh[0], bl[0]) + __hiloint2double(bh[1], bl[1]);
}

// Loop kernel: the divergence of the current links U_mu(x) = H(x) U0_mu(x) H(x+mu)^dag to D and one
// FP64 partial (F, theta) per block of 64 sites. Four lanes per site, one direction each: a wave covers
// 16 consecutive sites x 4 directions, so every load and store is a 16-site run in one plane. Lane mu
// forms U_mu(x) and the back neighbour's U_mu(x - mu) (the divergence needs both; neither is stored);
// all loads are issued before any arithmetic, so a wave waits for one memory round trip per site block.
// Per site it reads the four U0 links and H (736 B in FP64-18) and writes Delta (64 B).
//
// Traversals (autotuned per shape and precision; partials are stored by site block, so every traversal
// gives the same bits):
//  zb >= 1  one block per site block. The blocks sweep each (x, y) plane; with zb > 1 (zb divides Nz,
//           64 divides the plane) the planes are visited with z in groups of zb inside the t loop,
//           (z mod zb, t, z / zb), so that a site's t neighbour was read zb planes earlier and may still
//           be in the XCD's L2.
//  zb == 0  t-march: one block per 64-site run of the (x, y, z) volume, stepping through t. The lane of
//           direction t keeps the anti-Hermitian part of its own U_t from the previous step, which is
//           the U_t(x - t) of this one, so U0_t(x - t) and H(x - t) are never fetched again (except at
//           the block's first step). The blocks of one XCD (consecutive runs, xcd_remap) hold a slab of
//           the (x, y, z) volume and step through t together, so the y and z neighbours they read are in
//           that XCD's L2. Needs Nx Ny Nz to be a multiple of 64.
constexpr int kFusedThreads = 256;
constexpr int kFusedSites = kFusedThreads / 4;

// Element at a 32-bit byte offset from a wave-uniform base: the scalar-base form of the global memory
// instructions, one offset register per lane for every plane instead of a 64-bit address per load.
template <typename T>
__device__ __forceinline__ T ld_off(const T* base, uint32_t off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + off);
}
template <typename T>
__device__ __forceinline__ void st_off(T* base, uint32_t off, const T& v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off) = v;
}

template <typename T, int NE>
struct LoopIO {
    Links<T, NE> U0;
    const cx<T>* __restrict__ H;
    cx<T>* __restrict__ D;
    size_t ps;
};

// One site block: site s of this lane (valid if inside the lattice), direction mu. With keep set
// (t-march), the lane of direction t stores its own anti-Hermitian part there (an LDS slot of its site),
// and with reuse (after the block's first step) it takes the back neighbour's from there first. Returns
// this block's partial sums in thread 0. O32: the arrays of U0 and H span less than 4 GiB, so every
// load takes a 32-bit byte offset from the array's base (one register per lane and array instead of a
// 64-bit address). Measured: the FP64-18 sweep fits 128 VGPRs with it (four waves per SIMD instead of
// three) but runs no faster at 32^4; the float sweep at 32^3 x 64 went from 189 to 183 us.
template <typename T, int NE, bool O32>
__device__ __forceinline__ void loop_site_block(const LoopIO<T, NE>& io, const Geom& g, int64_t s, bool valid,
                                                int mu, bool reuse, AhAcc<T>* keep, double& fsum,
                                                double& tsum) {
    const size_t ps = io.ps;
    fsum = 0.0;
    tsum = 0.0;
    AhAcc<T> acc;
    acc.zero();
    if (valid) {
        int c[4];
        site_coords(g, s, c);
        // extents as wave-uniform values first: a select among fields of g by the per-lane mu would be
        // turned into a per-lane indexed load, which puts a copy of g in scratch memory
        const int n0 = __builtin_amdgcn_readfirstlane(g.n[0]), n1 = __builtin_amdgcn_readfirstlane(g.n[1]);
        const int n2 = __builtin_amdgcn_readfirstlane(g.n[2]), n3 = __builtin_amdgcn_readfirstlane(g.n[3]);
        const int cm = mu == 0 ? c[0] : mu == 1 ? c[1] : mu == 2 ? c[2] : c[3];
        const int nm = mu == 0 ? n0 : mu == 1 ? n1 : mu == 2 ? n2 : n3;
        const int64_t sm = mu == 0 ? 1 : mu == 1 ? (int64_t)n0 : mu == 2 ? (int64_t)n0 * n1 : (int64_t)n0 * n1 * n2;
        const int64_t sfw = cm == nm - 1 ? s - (int64_t)(nm - 1) * sm : s + sm;
        const int64_t sbk = cm == 0 ? s + (int64_t)(nm - 1) * sm : s - sm;
        // every load first; a lane that reuses its kept back neighbour reads its own site instead (lines
        // already on their way for its own link and H, so no extra traffic, and no branch around the loads)
        const int64_t sld = reuse ? s : sbk;
        su3<T> h0, hfw, hb, u, ub;
        if constexpr (O32) {
            constexpr uint32_t E = sizeof(cx<T>);
            const uint32_t oh0 = tile_byte_offset<cx<T>>(6, (uint32_t)s);
            const uint32_t ohf = tile_byte_offset<cx<T>>(6, (uint32_t)sfw);
            const uint32_t ohb = tile_byte_offset<cx<T>>(6, (uint32_t)sld);
            const uint32_t om = (uint32_t)(mu * NE * kTileSites) * E;
            const uint32_t ou0 = tile_byte_offset<cx<T>>(4 * NE, (uint32_t)s) + om;
            const uint32_t oub = tile_byte_offset<cx<T>>(4 * NE, (uint32_t)sld) + om;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                h0.e[k / 3][k % 3] = ld_off(io.H + k * kTileSites, oh0);
                hfw.e[k / 3][k % 3] = ld_off(io.H + k * kTileSites, ohf);
                hb.e[k / 3][k % 3] = ld_off(io.H + k * kTileSites, ohb);
            }
#pragma unroll
            for (int k = 0; k < NE; ++k) {
                u.e[k / 3][k % 3] = ld_off(io.U0.p + k * kTileSites, ou0);
                ub.e[k / 3][k % 3] = ld_off(io.U0.p + k * kTileSites, oub);
            }
        } else {
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                h0.e[k / 3][k % 3] = io.H[tile_index(6, k, s)];
                hfw.e[k / 3][k % 3] = io.H[tile_index(6, k, sfw)];
                hb.e[k / 3][k % 3] = io.H[tile_index(6, k, sld)];
            }
#pragma unroll
            for (int k = 0; k < NE; ++k) {
                u.e[k / 3][k % 3] = io.U0.p[io.U0.at(mu, k, s)];
                ub.e[k / 3][k % 3] = io.U0.p[io.U0.at(mu, k, sld)];
            }
        }
        third_row(h0.e[0], h0.e[1], h0.e[2]);
        third_row(hfw.e[0], hfw.e[1], hfw.e[2]);
        third_row(hb.e[0], hb.e[1], hb.e[2]);
        if constexpr (NE == 6) {
            third_row(u.e[0], u.e[1], u.e[2]);
            third_row(ub.e[0], ub.e[1], ub.e[2]);
        }
        const su3<T> un = updated_link(h0, u, hfw);  // U_mu(x)
        fsum = (double)un.e[0][0].re + (double)un.e[1][1].re + (double)un.e[2][2].re;
        AhAcc<T> own;
        own.set(un);
        acc.set(updated_link(hb, ub, h0));  // U_mu(x - mu)
        if (reuse) acc = *keep;
        acc.sub(own);
        if (keep != nullptr && mu == 3) *keep = own;
    }
    acc.o01.re = xor_sum4(acc.o01.re);
    acc.o01.im = xor_sum4(acc.o01.im);
    acc.o02.re = xor_sum4(acc.o02.re);
    acc.o02.im = xor_sum4(acc.o02.im);
    acc.o12.re = xor_sum4(acc.o12.re);
    acc.o12.im = xor_sum4(acc.o12.im);
    acc.d0 = xor_sum4(acc.d0);
    acc.d1 = xor_sum4(acc.d1);
    acc.d2 = xor_sum4(acc.d2);
    if (valid) {
        const T tr = (acc.d0 + acc.d1 + acc.d2) / T(3);
        const T d0 = T(2) * (acc.d0 - tr), d1 = T(2) * (acc.d1 - tr);
        const cx<T> z0 = acc.o01, z1 = acc.o02, z2 = acc.o12;
        const cx<T> out = mu == 0 ? z0 : mu == 1 ? z1 : mu == 2 ? z2 : cx<T>{d0, d1};
        // plain stores: D is read again by the (x, y) pass right after this kernel
        io.D[(size_t)mu * ps + s] = out;
        if (mu == 0) {
            const double e0 = norm2(z0), e1 = norm2(z1), e2 = norm2(z2);
            const double dd0 = d0, dd1 = d1;
            tsum = 2.0 * (e0 + e1 + e2) + dd0 * dd0 + dd1 * dd1 + (dd0 + dd1) * (dd0 + dd1);
        }
    }
    block_sum2<kFusedThreads>(fsum, tsum);
}

// force: measure even when the control block says the loop has stopped (a standalone measurement).
// TM: the t-march traversal (zb is then ignored); its own instantiation, so that the other traversals
// keep their register budget. O32: 32-bit load offsets (arrays below 4 GiB).
template <typename T, int NE, bool TM, bool O32>
__global__ void __launch_bounds__(kFusedThreads, 2) k_update_measure(Links<T, NE> U0, const cx<T>* __restrict__ H,
                                                                     cx<T>* __restrict__ D, size_t ps, Geom g,
                                                                     double2* __restrict__ part, Ctl* ctl, Batch bt,
                                                                     int zb, int force) {
    LoopIO<T, NE> io{U0, H, D, ps};
    {
        const size_t bo = boff(bt);
        io.U0.p = bshift(io.U0.p, bo);
        io.H = bshift(io.H, bo);
        io.D = bshift(io.D, bo);
        part = bshift(part, bo);
        ctl = bshift(ctl, bo);
    }
    if (!force && ctl->done) return;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int lane = threadIdx.x & 63;
    const int mu = lane >> 4;
    const int in_block = (threadIdx.x >> 6) * 16 + (lane & 15);  // site of this lane within its site block
    double fsum, tsum;
    if constexpr (TM) {
        // block b owns spatial sites b*64 .. b*64 + 63 at every t
        __shared__ AhAcc<T> keep[kFusedSites];
        const int64_t vs = g.stride[3];
        const int sbt = (int)(vs / kFusedSites);  // site blocks per t slice
#pragma unroll 1
        for (int t = 0; t < g.n[3]; ++t) {
            const int64_t s = (int64_t)b * kFusedSites + in_block + vs * t;
            loop_site_block<T, NE, O32>(io, g, s, true, mu, t > 0 && mu == 3, &keep[in_block], fsum, tsum);
            if (threadIdx.x == 0) part[b + sbt * t] = make_double2(fsum, tsum);
            __syncthreads();  // the block sum's LDS slots are written again in the next step
        }
    } else {
        int sb = b;  // site block: sites sb*64 .. sb*64 + 63
        if (zb > 1) {
            const int bpp = (g.n[0] * g.n[1]) / kFusedSites;
            const int P = b / bpp, off = b - P * bpp;
            const int z = P % zb + zb * (P / (zb * g.n[3]));
            const int t = (P / zb) % g.n[3];
            sb = (z + g.n[2] * t) * bpp + off;
        }
        const int64_t s = (int64_t)sb * kFusedSites + in_block;
        loop_site_block<T, NE, O32>(io, g, s, s < g.vol, mu, false, nullptr, fsum, tsum);
        if (threadIdx.x == 0) part[sb] = make_double2(fsum, tsum);
    }
    if (threadIdx.x == 0 && b == 0) ctl->pending = 1;
}

// ------------------------------------------------ loop kernel, brick march
// Bricks of the (x, y, z) volume: whole x rows, by rows in y and bz planes in z (Nx*by a multiple of 64,
// so that every 64-site block of the canonical order lies in one brick), each stepping through a segment
// of lt values of t. Every lane (site, direction mu) forms the one link it owns, U_mu(x), and puts its
// anti-Hermitian part in LDS; the divergence at x then takes that of the back link U_mu(x - mu) from the
// lane that owns it: the same brick at this step (x, and y or z inside the brick), the previous step
// (t), or a halo lane that forms the links entering the brick from below in y and z (and in t at the
// segment's first step). Links are formed once each instead of twice, and the back links' U0 and H are
// fetched only for the halo. The arithmetic of every link and of the divergence is that of the other
// traversals and the partials are summed by 64-site block in the same order, so the results are the
// same bits.
struct BrickGeom {
    int by, bz;    // rows in y, planes in z per brick
    int nby, nbz;  // bricks along y and z
    int lt;        // t steps per segment
};

// Nine planes of n anti-Hermitian parts in LDS (structure of arrays).
template <typename T>
struct AhPlanes {
    T* p;
    int n;
    __device__ __forceinline__ void put(int i, const AhAcc<T>& a) const {
        p[i] = a.o01.re;
        p[n + i] = a.o01.im;
        p[2 * n + i] = a.o02.re;
        p[3 * n + i] = a.o02.im;
        p[4 * n + i] = a.o12.re;
        p[5 * n + i] = a.o12.im;
        p[6 * n + i] = a.d0;
        p[7 * n + i] = a.d1;
        p[8 * n + i] = a.d2;
    }
    __device__ __forceinline__ AhAcc<T> get(int i) const {
        AhAcc<T> a;
        a.o01 = {p[i], p[n + i]};
        a.o02 = {p[2 * n + i], p[3 * n + i]};
        a.o12 = {p[4 * n + i], p[5 * n + i]};
        a.d0 = p[6 * n + i];
        a.d1 = p[7 * n + i];
        a.d2 = p[8 * n + i];
        return a;
    }
};

// Anti-Hermitian part of U_m(xb) = H(xb) U0_m(xb) H(x)^dag, xb the back neighbour of x along m (site
// indices below 2^32 / 16; the caller checks the lattice fits).
template <typename T, int NE>
__device__ __forceinline__ AhAcc<T> back_link_ah(const LoopIO<T, NE>& io, int m, uint32_t x, uint32_t xb) {
    constexpr uint32_t E = sizeof(cx<T>);
    su3<T> hb, ub, h0;
    const uint32_t ob = tile_byte_offset<cx<T>>(6, xb), ox = tile_byte_offset<cx<T>>(6, x);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        hb.e[k / 3][k % 3] = ld_off(io.H + k * kTileSites, ob);
        h0.e[k / 3][k % 3] = ld_off(io.H + k * kTileSites, ox);
    }
    const uint32_t ou = tile_byte_offset<cx<T>>(4 * NE, xb) + (uint32_t)(m * NE * kTileSites) * E;
#pragma unroll
    for (int k = 0; k < NE; ++k) ub.e[k / 3][k % 3] = ld_off(io.U0.p + k * kTileSites, ou);
    third_row(hb.e[0], hb.e[1], hb.e[2]);
    third_row(h0.e[0], h0.e[1], h0.e[2]);
    if constexpr (NE == 6) third_row(ub.e[0], ub.e[1], ub.e[2]);
    AhAcc<T> a;
    a.set(updated_link(hb, ub, h0));
    return a;
}

// LDS bytes of one brick: own links (4 per site), the previous step's t links, the y and z halos.
__host__ __device__ constexpr size_t brick_lds(int nx, int ny, int nz, int by, int bz, size_t tsz) {
    return (size_t)9 * tsz *
           (5 * (size_t)nx * by * bz + (by < ny ? (size_t)nx * bz : 0) + (bz < nz ? (size_t)nx * by : 0));
}

// NTB = 4 * Nx * by * bz threads; grid = bricks * segments.
template <typename T, int NE, int NTB>
__global__ void __launch_bounds__(NTB) k_update_measure_brick(Links<T, NE> U0, const cx<T>* __restrict__ H,
                                                              cx<T>* __restrict__ D, size_t ps, Geom g,
                                                              BrickGeom bg, double2* __restrict__ part, Ctl* ctl,
                                                              Batch bt, int force) {
    LoopIO<T, NE> io{U0, H, D, ps};
    {
        const size_t bo = boff(bt);
        io.U0.p = bshift(io.U0.p, bo);
        io.H = bshift(io.H, bo);
        io.D = bshift(io.D, bo);
        part = bshift(part, bo);
        ctl = bshift(ctl, bo);
    }
    if (!force && ctl->done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double sa[NTB / 64], sb[NTB / 64];
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2], nt = g.n[3];
    const int R = NTB / 4;  // sites per brick
    const int hy = bg.by < ny ? nx * bg.bz : 0, hz = bg.bz < nz ? nx * bg.by : 0;
    T* lds = reinterpret_cast<T*>(smem);
    // LDS planes: own links (entry mu * R + r), the previous step's t links (R), y halo (hy), z halo (hz)
    const AhPlanes<T> own{lds, 4 * R};
    const AhPlanes<T> prev{lds + 9 * 4 * R, R};

    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int nbr = bg.nby * bg.nbz;
    const int brick = b % nbr, seg = b / nbr;
    const int y0 = (brick % bg.nby) * bg.by, z0 = (brick / bg.nby) * bg.bz;
    const int t0 = seg * bg.lt;
    const int64_t sy = nx, sz = (int64_t)nx * ny, vs = sz * nz;

    const int lane = threadIdx.x & 63;
    const int mu = lane >> 4;
    const int r = (threadIdx.x >> 6) * 16 + (lane & 15);  // brick site of this lane
    const int xl = r % nx, yl = (r / nx) % bg.by, zl = r / (nx * bg.by);
    const int64_t sxy = xl + sy * (y0 + yl) + sz * (z0 + zl);
    const int cm = mu == 0 ? xl : mu == 1 ? y0 + yl : z0 + zl;  // coordinate along mu (spatial mu)
    const int nm = mu == 0 ? nx : mu == 1 ? ny : nz;
    const int64_t sm = mu == 0 ? 1 : mu == 1 ? sy : sz;
    const int64_t dfw_sp = cm == nm - 1 ? -(int64_t)(nm - 1) * sm : sm;
    // where this lane finds the anti-Hermitian part of its back link: planes (offset in T, length) and
    // slot; one read through a per-lane choice of planes, not one read per source
    int bk_off = 0, bk_n = 4 * R, bk_i = 0;
    if (mu == 0) {
        bk_i = xl == 0 ? r + nx - 1 : r - 1;
    } else if (mu == 1) {
        if (yl > 0) bk_i = R + r - nx;
        else if (hy == 0) bk_i = R + r + nx * (bg.by - 1);
        else {
            bk_off = 9 * 5 * R;
            bk_n = hy;
            bk_i = xl + nx * zl;
        }
    } else if (mu == 2) {
        if (zl > 0) bk_i = 2 * R + r - nx * bg.by;
        else if (hz == 0) bk_i = 2 * R + r + nx * bg.by * (bg.bz - 1);
        else {
            bk_off = 9 * (5 * R + hy);
            bk_n = hz;
            bk_i = xl + nx * yl;
        }
    } else {
        bk_off = 9 * 4 * R;
        bk_n = R;
        bk_i = r;
    }
    const AhPlanes<T> back{lds + bk_off, bk_n};
    // this thread's halo task: a y, z or (first step) t link entering the brick from below
    const int task = threadIdx.x;
    int hm = 0;
    int64_t hxy = 0, hdb = 0;  // halo site (spatial) and the offset to its back neighbour
    int hslot = 0, h_off = 0, h_n = 1;
    if (task < hy) {
        hm = 1;
        const int hx = task % nx, hzl = task / nx;
        hxy = hx + sy * y0 + sz * (z0 + hzl);
        hdb = y0 == 0 ? (int64_t)(ny - 1) * sy : -sy;
        hslot = task;
        h_off = 9 * 5 * R;
        h_n = hy;
    } else if (task < hy + hz) {
        hm = 2;
        const int j = task - hy;
        const int hx = j % nx, hyl = j / nx;
        hxy = hx + sy * (y0 + hyl) + sz * z0;
        hdb = z0 == 0 ? (int64_t)(nz - 1) * sz : -sz;
        hslot = j;
        h_off = 9 * (5 * R + hy);
        h_n = hz;
    } else if (task < hy + hz + R) {
        hm = 3;  // first step only
        const int j = task - hy - hz;
        const int jx = j % nx, jy = (j / nx) % bg.by, jz = j / (nx * bg.by);
        hxy = jx + sy * (y0 + jy) + sz * (z0 + jz);
        hdb = t0 == 0 ? (int64_t)(nt - 1) * vs : -vs;
        hslot = j;
        h_off = 9 * 4 * R;
        h_n = R;
    }
    const AhPlanes<T> hdst{lds + h_off, h_n};
    const int gi = threadIdx.x >> 8;  // 64-site block of this thread within the brick
#pragma unroll 1
    for (int tt = t0; tt < t0 + bg.lt; ++tt) {
        // t through a wave-uniform intrinsic: addresses are recomputed from it each step rather than
        // carried as one induction pointer per load (which took the registers of a second wave)
        const int t = __builtin_amdgcn_readfirstlane(tt);
        // the halo first, so that none of this lane's own link is held meanwhile
        if (hm == 1 || hm == 2 || (hm == 3 && t == t0)) {
            const int64_t hs = hxy + vs * t;
            hdst.put(hslot, back_link_ah<T, NE>(io, hm, (uint32_t)hs, (uint32_t)(hs + hdb)));
        }
        const int64_t s = sxy + vs * t;
        const int64_t sfw = mu == 3 ? (t == nt - 1 ? s - (int64_t)(nt - 1) * vs : s + vs) : s + dfw_sp;
        constexpr uint32_t E = sizeof(cx<T>);
        const uint32_t os = tile_byte_offset<cx<T>>(6, (uint32_t)s), ofw = tile_byte_offset<cx<T>>(6, (uint32_t)sfw);
        const uint32_t ou = tile_byte_offset<cx<T>>(4 * NE, (uint32_t)s) + (uint32_t)(mu * NE * kTileSites) * E;
        su3<T> h0, hfw, u;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            h0.e[k / 3][k % 3] = ld_off(io.H + k * kTileSites, os);
            hfw.e[k / 3][k % 3] = ld_off(io.H + k * kTileSites, ofw);
        }
#pragma unroll
        for (int k = 0; k < NE; ++k) u.e[k / 3][k % 3] = ld_off(io.U0.p + k * kTileSites, ou);
        third_row(h0.e[0], h0.e[1], h0.e[2]);
        third_row(hfw.e[0], hfw.e[1], hfw.e[2]);
        if constexpr (NE == 6) third_row(u.e[0], u.e[1], u.e[2]);
        const su3<T> un = updated_link(h0, u, hfw);  // U_mu(x)
        double fsum = (double)un.e[0][0].re + (double)un.e[1][1].re + (double)un.e[2][2].re;
        AhAcc<T> mine;
        mine.set(un);
        own.put(mu * R + r, mine);
        __syncthreads();
        AhAcc<T> acc = back.get(bk_i);
        acc.sub(mine);
        if (mu == 3) prev.put(r, mine);  // the back t link of the next step (only this lane uses the slot)
        acc.o01.re = xor_sum4(acc.o01.re);
        acc.o01.im = xor_sum4(acc.o01.im);
        acc.o02.re = xor_sum4(acc.o02.re);
        acc.o02.im = xor_sum4(acc.o02.im);
        acc.o12.re = xor_sum4(acc.o12.re);
        acc.o12.im = xor_sum4(acc.o12.im);
        acc.d0 = xor_sum4(acc.d0);
        acc.d1 = xor_sum4(acc.d1);
        acc.d2 = xor_sum4(acc.d2);
        double tsum = 0.0;
        {
            const T tr = (acc.d0 + acc.d1 + acc.d2) / T(3);
            const T d0 = T(2) * (acc.d0 - tr), d1 = T(2) * (acc.d1 - tr);
            const cx<T> z0c = acc.o01, z1c = acc.o02, z2c = acc.o12;
            const cx<T> out = mu == 0 ? z0c : mu == 1 ? z1c : mu == 2 ? z2c : cx<T>{d0, d1};
            st_off(io.D, ((uint32_t)mu * (uint32_t)ps + (uint32_t)s) * E, out);
            if (mu == 0) {
                const double e0 = norm2(z0c), e1 = norm2(z1c), e2 = norm2(z2c);
                const double dd0 = d0, dd1 = d1;
                tsum = 2.0 * (e0 + e1 + e2) + dd0 * dd0 + dd1 * dd1 + (dd0 + dd1) * (dd0 + dd1);
            }
        }
        // partial sums of each 64-site block (four waves, in the order of the other traversals)
        fsum = wave_sum(fsum);
        tsum = wave_sum(tsum);
        if (lane == 0) {
            sa[threadIdx.x >> 6] = fsum;
            sb[threadIdx.x >> 6] = tsum;
        }
        __syncthreads();
        if ((threadIdx.x & 255) == 0) {
            double ta = 0.0, tb = 0.0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                ta += sa[4 * gi + i];
                tb += sb[4 * gi + i];
            }
            part[s / kFusedSites] = make_double2(ta, tb);  // this thread's site opens the 64-site block
        }
    }
    if (threadIdx.x == 0 && blockIdx.x == 0) ctl->pending = 1;
}

// ------------------------------------------------ mixed-precision hand-over
// Rows 1-2 of the identity in the six planes of a transform.
template <typename T>
__global__ void __launch_bounds__(kSiteThreads) k_gauge_identity(cx<T>* __restrict__ A, int64_t vol) {
    const int64_t s = (int64_t)blockIdx.x * kSiteThreads + threadIdx.x;
    if (s >= vol) return;
#pragma unroll
    for (int k = 0; k < 6; ++k) A[tile_index(6, k, s)] = {(k == 0 || k == 4) ? T(1) : T(0), T(0)};
}

// The float transform accumulated by the bulk iterations, promoted to double and re-orthonormalised in
// double: the double-precision phase continues from the same links, H U0 H(x+mu)^dag, with U0 the
// untouched input in double.
__global__ void __launch_bounds__(kSiteThreads) k_promote_h(const cx<float>* __restrict__ A, cx<double>* __restrict__ B,
                                                            int64_t vol) {
    const int64_t s = (int64_t)blockIdx.x * kSiteThreads + threadIdx.x;
    if (s >= vol) return;
    su3<double> m;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const cx<float> e = A[tile_index(6, k, s)];
        m.e[k / 3][k % 3] = {(double)e.re, (double)e.im};
    }
    reunitarize(m);
#pragma unroll
    for (int k = 0; k < 6; ++k) B[tile_index(6, k, s)] = m.e[k / 3][k % 3];
}

// --------------------------------------------------------------------- FFT
// 2D FFT over the (x, y) plane, src -> dst (may alias). Each block takes G
// consecutive planes of one field (flattened plane index = field * Nz*Nt +
// z + Nz*t), stages them in LDS with rows padded to rs elements, transforms
// along x then y, and writes them out. With part set and first true, the block
// first reduces the loop kernel's pending partials (npart of them) into the
// control block (the fused batch's first block of a configuration; the
// per-shape kernels give the reduction a block of its own).
template <typename T, int EPT, bool INV>
__device__ __forceinline__ void fft_xy_body(const cx<T>* src, cx<T>* dst, size_t zps, int nx, int ny, int nzt,
                                            int G, int rs, const FftPlan& px, const FftPlan& py,
                                            const cx<T>* __restrict__ twgx, const cx<T>* __restrict__ twgy,
                                            Ctl* ctl, int force, const double2* __restrict__ part, int npart,
                                            double inv3v, double inv12v, int blk, bool first) {
    if (part != nullptr && first && ctl->pending) {
        reduce_partials(part, npart, inv3v, inv12v, ctl, 1);
        __syncthreads();
    }
    if (!force && ctl->done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T>* twx = reinterpret_cast<cx<T>*>(smem);
    cx<T>* twy = twx + nx;
    cx<T>* buf = twy + ny;
    const int nthr = blockDim.x;
    for (int i = threadIdx.x; i < nx; i += nthr) twx[i] = twgx[i];
    for (int i = threadIdx.x; i < ny; i += nthr) twy[i] = twgy[i];
    const int q0 = blk * G;
    const int f = q0 / nzt, zt0 = q0 - f * nzt;
    const size_t off = (size_t)f * zps + (size_t)zt0 * nx * ny;
    const cx<T>* gs = src + off;
    cx<T>* gd = dst + off;
    const int E = G * nx * ny;
    for (int e = threadIdx.x; e < E; e += nthr) {
        const int row = e / nx, x = e - row * nx;
        buf[row * rs + x] = gs[e];
    }
    __syncthreads();
    fft_rows<EPT, T, INV>(buf, twx, px, 1, G * ny, G * ny, rs, 0);
    fft_rows<EPT, T, INV>(buf, twy, py, rs, G * nx, nx, 1, ny * rs);
    for (int e = threadIdx.x; e < E; e += nthr) {
        const int row = e / nx, x = e - row * nx;
        gd[e] = buf[row * rs + x];
    }
}

template <typename T, int EPT, bool INV>
__global__ void __launch_bounds__(1024) k_fft_xy(const cx<T>* src, cx<T>* dst, size_t zps, int nx, int ny,
                                                 int nzt, int G, int rs, FftPlan px, FftPlan py,
                                                 const cx<T>* __restrict__ twgx, const cx<T>* __restrict__ twgy,
                                                 Ctl* ctl, int force, const double2* __restrict__ part, int npart,
                                                 double inv3v, double inv12v, Batch bt) {
    {
        const size_t bo = boff(bt);
        src = bshift(src, bo);
        dst = bshift(dst, bo);
        twgx = bshift(twgx, bo);
        twgy = bshift(twgy, bo);
        ctl = bshift(ctl, bo);
        part = bshift(part, bo);
    }
    // With part set, block 0 (dispatched first) only reduces the pending partials; the others transform.
    const int red = part != nullptr ? 1 : 0;
    if (red && blockIdx.x == 0) {
        if (ctl->pending) reduce_partials(part, npart, inv3v, inv12v, ctl, 1);
        return;
    }
    fft_xy_body<T, EPT, INV>(src, dst, zps, nx, ny, nzt, G, rs, px, py, twgx, twgy, ctl, force, nullptr, 0, inv3v,
                             inv12v, xcd_remap(blockIdx.x - red, gridDim.x - red), false);
}

// 2D FFT over (z, t), filter and inverse (z, t) of block blk's bx columns (the body of k_fft_zt).
template <typename T, int EPT>
__device__ __forceinline__ void fft_zt_body(cx<T>* __restrict__ Z, size_t zps, int nx, int ny, int nz, int nt,
                                            int bx, int tsp, const FftPlan& pz, const FftPlan& pt,
                                            const cx<T>* __restrict__ twgz, const cx<T>* __restrict__ twgt,
                                            const T* __restrict__ sin2, T coef, int no_fa,
                                            const Ctl* __restrict__ ctl, int force, const T* __restrict__ mtab,
                                            const TupleGeom& tg, cx<T>* __restrict__ spec, int blk) {
    if (!force && ctl->done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T>* twz = reinterpret_cast<cx<T>*>(smem);
    cx<T>* twt = twz + nz;
    cx<T>* buf = twt + nt;
    const int nthr = blockDim.x;
    for (int i = threadIdx.x; i < nz; i += nthr) twz[i] = twgz[i];
    for (int i = threadIdx.x; i < nt; i += nthr) twt[i] = twgt[i];
    const int nxb = nx / bx;
    const int xb = blk % nxb;
    const int rest = blk / nxb;
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
        const int li = t * tsp + z * bx + xo;
        if (spec) spec[xo + zt * pstep + (gp - Z)] = buf[li];
        T mult;
        if (mtab) {
            mult = mtab[tuple_index(tg, x0 + xo, y, z, t)];
        } else {
            const T p2 = sx[x0 + xo] + sy[y] + sz[z] + st[t];
            mult = p2 > T(0) ? (no_fa ? coef : coef / p2) : T(0);
        }
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

// 2D FFT over (z, t) for bx consecutive x columns at one y of one field,
// multiply every mode by coef / p^2(p) (coef = (alpha/2) p2max / V; zero mode
// -> 0; coef alone when no_fa), then the inverse (z, t) transform, in place.
// LDS element (xo, z, t) sits at t*tsp + z*bx + xo.
template <typename T, int EPT>
__global__ void __launch_bounds__(1024) k_fft_zt(cx<T>* __restrict__ Z, size_t zps, int nx, int ny, int nz, int nt,
                                                 int bx, int tsp, FftPlan pz, FftPlan pt,
                                                 const cx<T>* __restrict__ twgz, const cx<T>* __restrict__ twgt,
                                                 const T* __restrict__ sin2, T coef, int no_fa,
                                                 const Ctl* __restrict__ ctl, int force, const T* __restrict__ mtab,
                                                 TupleGeom tg, cx<T>* __restrict__ spec, Batch bt) {
    {
        const size_t bo = boff(bt);
        Z = bshift(Z, bo);
        twgz = bshift(twgz, bo);
        twgt = bshift(twgt, bo);
        sin2 = bshift(sin2, bo);
        ctl = bshift(ctl, bo);
    }
    fft_zt_body<T, EPT>(Z, zps, nx, ny, nz, nt, bx, tsp, pz, pt, twgz, twgt, sin2, coef, no_fa, ctl, force, mtab, tg,
                        spec, xcd_remap(blockIdx.x, gridDim.x));
}

// Inverse 2D FFT over (x, y) of all four packed fields of one (z, t) plane,
// then g(x) = reunitarize(1 + (alpha/2) Delta~(x)) for every site of the
// plane and the update of the stored transform, Hout = reunitarize(g Hin)
// (rows 1-2, in tiles of 64 sites); with Hin null, g itself goes to Hout.
template <typename T, int EPT>
__device__ __forceinline__ void fft_xy_gauge_body(const cx<T>* __restrict__ Q, size_t zps,
                                                  const cx<T>* __restrict__ Hin, cx<T>* __restrict__ Hout,
                                                  int nx, int ny, int rs, const FftPlan& px,
                                                  const FftPlan& py, const cx<T>* __restrict__ twgx,
                                                  const cx<T>* __restrict__ twgy, const Ctl* __restrict__ ctl,
                                                  int force, int exact, int blk) {
    if (!force && ctl->done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T>* twx = reinterpret_cast<cx<T>*>(smem);
    cx<T>* twy = twx + nx;
    cx<T>* buf = twy + ny;
    const int nthr = blockDim.x;
    for (int i = threadIdx.x; i < nx; i += nthr) twx[i] = twgx[i];
    for (int i = threadIdx.x; i < ny; i += nthr) twy[i] = twgy[i];
    const int P = nx * ny;
    const int pl = ny * rs;  // LDS elements per field plane
    const size_t base = (size_t)blk * P;
    for (int e = threadIdx.x; e < 4 * P; e += nthr) {
        const int f = e / P, r = e - f * P;
        const int row = r / nx, x = r - row * nx;
        buf[f * pl + row * rs + x] = Q[(size_t)f * zps + base + r];
    }
    __syncthreads();
    fft_rows<EPT, T, true>(buf, twx, px, 1, 4 * ny, 4 * ny, rs, 0);
    fft_rows<EPT, T, true>(buf, twy, py, rs, 4 * nx, nx, 1, pl);
    for (int r = threadIdx.x; r < P; r += nthr) {
        const int row = r / nx, x = r - row * nx;
        const int li = row * rs + x;
        su3<T> g = g_from_packed(buf[li], buf[pl + li], buf[2 * pl + li], buf[3 * pl + li], exact != 0);
        if (Hin != nullptr) {
            su3<T> h;
#pragma unroll
            for (int k = 0; k < 6; ++k) h.e[k / 3][k % 3] = Hin[tile_index(6, k, base + r)];
            g = gauge_times(g, h);
        }
#pragma unroll
        for (int k = 0; k < 6; ++k) Hout[tile_index(6, k, base + r)] = g.e[k / 3][k % 3];
    }
}

template <typename T, int EPT>
__global__ void __launch_bounds__(EPT == 16 ? 640 : 1024) k_fft_xy_gauge(const cx<T>* __restrict__ Q, size_t zps,
                                                       const cx<T>* __restrict__ Hin, cx<T>* __restrict__ Hout,
                                                       int nx, int ny, int rs, FftPlan px, FftPlan py,
                                                       const cx<T>* __restrict__ twgx, const cx<T>* __restrict__ twgy,
                                                       const Ctl* __restrict__ ctl, int force, Batch bt, int exact) {
    {
        const size_t bo = boff(bt);
        Q = bshift(Q, bo);
        Hin = bshift(Hin, bo);
        Hout = bshift(Hout, bo);
        twgx = bshift(twgx, bo);
        twgy = bshift(twgy, bo);
        ctl = bshift(ctl, bo);
    }
    fft_xy_gauge_body<T, EPT>(Q, zps, Hin, Hout, nx, ny, rs, px, py, twgx, twgy, ctl, force, exact,
                              xcd_remap(blockIdx.x, gridDim.x));
}

}  // namespace gf

// Device-side building blocks for libgf: complex arithmetic, SU(3) algebra,
// link storage access, site geometry and block reductions (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gf {

// ------------------------------------------------------------------ complex
template <typename T>
struct cx {
    T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
// Every product of two complex numbers is written with explicit fused multiply-adds (one product
// rounded, the other fused), so no result depends on where the compiler chooses to contract: the loop
// kernel forms the same updated link at two places (a lane's own link, and the back neighbour's link
// for the divergence) and needs both to give the same bits.
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re)};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
    return {fma(a.re, b.re, a.im * b.im), fma(a.im, b.re, -(a.re * b.im))};
}
// conj(a) * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulcc(cx<T> a, cx<T> b) {
    return {fma(a.re, b.re, -(a.im * b.im)), -fma(a.re, b.im, a.im * b.re)};
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T>
__device__ __forceinline__ T norm2(cx<T> a) { return fma(a.re, a.re, a.im * a.im); }
// acc + a*b
template <typename T>
__device__ __forceinline__ cx<T> cfma(cx<T> acc, cx<T> a, cx<T> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
    return acc;
}
// acc + a*conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cfmac(cx<T> acc, cx<T> a, cx<T> b) {
    acc.re = fma(a.re, b.re, acc.re);
    acc.re = fma(a.im, b.im, acc.re);
    acc.im = fma(a.im, b.re, acc.im);
    acc.im = fma(-a.re, b.im, acc.im);
    return acc;
}

__device__ __forceinline__ double inv_sqrt(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float inv_sqrt(float x) { return __frsqrt_rn(x); }

// Streaming stores (and loads) with the nontemporal hint: the loop kernel writes the updated links and
// the divergence once and reads them again only in a later launch, and the link field is larger than
// the last-level cache, so keeping those lines cached only evicts reusable ones (measured: 4-6 % off
// the loop kernel at 32^4 in every precision).
template <typename T>
__device__ __forceinline__ void nt_store(cx<T>* p, cx<T> v) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    v2 x = {v.re, v.im};
    __builtin_nontemporal_store(x, reinterpret_cast<v2*>(p));
}
template <typename T>
__device__ __forceinline__ cx<T> nt_load(const cx<T>* p) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 x = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
    return {x.x, x.y};
}

// ------------------------------------------------------------------- SU(3)
template <typename T>
struct su3 {
    cx<T> e[3][3];
};

// Row 3 of an SU(3) matrix from rows 1 and 2: r3 = conj(r1 x r2).
template <typename T>
__device__ __forceinline__ void third_row(const cx<T>* r1, const cx<T>* r2, cx<T>* r3) {
    r3[0] = conj(cmul(r1[1], r2[2]) - cmul(r1[2], r2[1]));
    r3[1] = conj(cmul(r1[2], r2[0]) - cmul(r1[0], r2[2]));
    r3[2] = conj(cmul(r1[0], r2[1]) - cmul(r1[1], r2[0]));
}

// 1/sqrt(x) in double from the hardware estimate and one Newton step, y (3 - x y^2) / 2, which squares its
// relative error: ample for results that are then rounded to float.
__device__ __forceinline__ double rsqrt_newton(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    return y * fma(-0.5 * x * y, y, 1.5);
}

// Row Gram-Schmidt onto SU(3): normalise r1, orthogonalise and normalise r2,
// rebuild r3 from unitarity and det = 1.
template <typename T>
__device__ __forceinline__ void reunitarize(su3<T>& m) {
    T n1 = norm2(m.e[0][0]) + norm2(m.e[0][1]) + norm2(m.e[0][2]);
    T i1 = inv_sqrt(n1);
#pragma unroll
    for (int j = 0; j < 3; ++j) m.e[0][j] = cscale(m.e[0][j], i1);
    cx<T> d = {T(0), T(0)};
#pragma unroll
    for (int j = 0; j < 3; ++j) d = cfma(d, conj(m.e[0][j]), m.e[1][j]);
#pragma unroll
    for (int j = 0; j < 3; ++j) m.e[1][j] = m.e[1][j] - cmul(d, m.e[0][j]);
    T n2 = norm2(m.e[1][0]) + norm2(m.e[1][1]) + norm2(m.e[1][2]);
    T i2 = inv_sqrt(n2);
#pragma unroll
    for (int j = 0; j < 3; ++j) m.e[1][j] = cscale(m.e[1][j], i2);
    third_row(m.e[0], m.e[1], m.e[2]);
}

// Row Gram-Schmidt in double precision whatever the storage type: rows 1-2 of a float matrix are
// promoted, orthonormalised in double and rounded back, and row 3 is rebuilt from them in float, so the
// bulk float iterations keep their reunitarisation in FP64.
template <typename T>
__device__ __forceinline__ void reunitarize_fp64(su3<T>& m) {
    if constexpr (sizeof(T) == 8) {
        reunitarize(m);
    } else {
        cx<double> r1[3], r2[3];
        double n1 = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            r1[j] = {(double)m.e[0][j].re, (double)m.e[0][j].im};
            r2[j] = {(double)m.e[1][j].re, (double)m.e[1][j].im};
            n1 += norm2(r1[j]);
        }
        const double i1 = rsqrt_newton(n1);
        cx<double> d = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            r1[j] = cscale(r1[j], i1);
            d = cfma(d, conj(r1[j]), r2[j]);
        }
        double n2 = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            r2[j] = r2[j] - cmul(d, r1[j]);
            n2 += norm2(r2[j]);
        }
        const double i2 = rsqrt_newton(n2);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            m.e[0][j] = {(T)r1[j].re, (T)r1[j].im};
            m.e[1][j] = {(T)(r2[j].re * i2), (T)(r2[j].im * i2)};
        }
        third_row(m.e[0], m.e[1], m.e[2]);
    }
}

// c = a * b
template <typename T>
__device__ __forceinline__ su3<T> mul(const su3<T>& a, const su3<T>& b) {
    su3<T> c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<T> s = cmul(a.e[i][0], b.e[0][j]);
            s = cfma(s, a.e[i][1], b.e[1][j]);
            s = cfma(s, a.e[i][2], b.e[2][j]);
            c.e[i][j] = s;
        }
    return c;
}

// c = a * b^dagger, rows 0..NR-1 of c only
template <typename T, int NR = 3>
__device__ __forceinline__ su3<T> mul_adj(const su3<T>& a, const su3<T>& b) {
    su3<T> c;
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<T> s = cmulc(a.e[i][0], b.e[j][0]);
            s = cfmac(s, a.e[i][1], b.e[j][1]);
            s = cfmac(s, a.e[i][2], b.e[j][2]);
            c.e[i][j] = s;
        }
    return c;
}

// rows 0..NR-1 of a * b
template <typename T, int NR>
__device__ __forceinline__ su3<T> mul_rows(const su3<T>& a, const su3<T>& b) {
    su3<T> c;
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<T> s = cmul(a.e[i][0], b.e[0][j]);
            s = cfma(s, a.e[i][1], b.e[1][j]);
            s = cfma(s, a.e[i][2], b.e[2][j]);
            c.e[i][j] = s;
        }
    return c;
}

// The link gl U gr^dag (gl, gr: the transform at x and at x + mu): rows 1-2 formed, row 3 rebuilt from
// unitarity. The loop kernel calls it for a lane's own link and for the back neighbour's link U_mu(x - mu);
// the same inlined code on the same operands gives the same bits as the neighbour's own result, so every
// traversal of the lattice computes the same divergence.
template <typename T>
__device__ __forceinline__ su3<T> updated_link(const su3<T>& gl, const su3<T>& u, const su3<T>& gr) {
    su3<T> un = mul_adj<T, 2>(mul_rows<T, 2>(gl, u), gr);
    third_row(un.e[0], un.e[1], un.e[2]);
    return un;
}

// exp(X) of an anti-Hermitian traceless 3x3 matrix in closed form (Cayley-Hamilton): with the
// Hermitian Q = -iX, c0 = det Q, c1 = Tr Q^2 / 2, theta = acos(|c0| / (2 (c1/3)^(3/2))),
// u = sqrt(c1/3) cos(theta/3), w = sqrt(c1) sin(theta/3), exp(iQ) = f0 + f1 Q + f2 Q^2 with
// f_j = h_j / (9u^2 - w^2),
//   h0 = (u^2 - w^2) e^{2iu} + e^{-iu} (8u^2 cos w + 2iu (3u^2 + w^2) xi0(w)),
//   h1 = 2u e^{2iu} - e^{-iu} (2u cos w - i (3u^2 - w^2) xi0(w)),
//   h2 = e^{2iu} - e^{-iu} (cos w + 3iu xi0(w)),  xi0(w) = sin(w)/w,
// and f_j -> (-1)^j conj(f_j) for c0 < 0 (Morningstar and Peardon, Phys. Rev. D 69 (2004) 054501).
// All terms of h_j are O(c1) or larger relative to the denominator, so small X keeps full precision.
template <typename T>
__device__ __forceinline__ su3<T> expm_su3(const su3<T>& X) {
    su3<T> Q;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Q.e[i][j] = {X.e[i][j].im, -X.e[i][j].re};
    T c1 = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) c1 += norm2(Q.e[i][j]);
    c1 *= T(0.5);
    su3<T> r;
    if (!(c1 > (sizeof(T) == 4 ? T(1e-30) : T(1e-200)))) {  // exp(X) = 1 + X to working precision
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) r.e[i][j] = {X.e[i][j].re + (i == j ? T(1) : T(0)), X.e[i][j].im};
        return r;
    }
    const cx<T> m0 = cmul(Q.e[1][1], Q.e[2][2]) - cmul(Q.e[1][2], Q.e[2][1]);
    const cx<T> m1 = cmul(Q.e[1][0], Q.e[2][2]) - cmul(Q.e[1][2], Q.e[2][0]);
    const cx<T> m2 = cmul(Q.e[1][0], Q.e[2][1]) - cmul(Q.e[1][1], Q.e[2][0]);
    const T c0 = (cmul(Q.e[0][0], m0) - cmul(Q.e[0][1], m1) + cmul(Q.e[0][2], m2)).re;
    const bool neg = c0 < T(0);
    const T c0max = T(2) * (c1 / T(3)) * sqrt(c1 / T(3));
    const T th = acos(fmin(fabs(c0) / c0max, T(1)));
    const T u = sqrt(c1 / T(3)) * cos(th / T(3));
    const T w = sqrt(c1) * sin(th / T(3));
    const T w2 = w * w, u2 = u * u;
    const T xi0 = fabs(w) < T(0.05) ? T(1) - w2 / T(6) * (T(1) - w2 / T(20) * (T(1) - w2 / T(42))) : sin(w) / w;
    const cx<T> e2 = {cos(T(2) * u), sin(T(2) * u)};
    const cx<T> em = {cos(u), -sin(u)};
    const T cw = cos(w);
    const cx<T> h0 = cscale(e2, u2 - w2) + cmul(em, cx<T>{T(8) * u2 * cw, T(2) * u * (T(3) * u2 + w2) * xi0});
    const cx<T> h1 = cscale(e2, T(2) * u) - cmul(em, cx<T>{T(2) * u * cw, -(T(3) * u2 - w2) * xi0});
    const cx<T> h2 = e2 - cmul(em, cx<T>{cw, T(3) * u * xi0});
    const T inv = T(1) / (T(9) * u2 - w2);
    cx<T> f0 = cscale(h0, inv), f1 = cscale(h1, inv), f2 = cscale(h2, inv);
    if (neg) {
        f0 = conj(f0);
        f1 = {-f1.re, f1.im};
        f2 = conj(f2);
    }
    const su3<T> Q2 = mul(Q, Q);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<T> v = cmul(f1, Q.e[i][j]) + cmul(f2, Q2.e[i][j]);
            if (i == j) v = v + f0;
            r.e[i][j] = v;
        }
    return r;
}

// g = reunitarize(1 + X), or of exp(X) if exact, X the anti-Hermitian traceless matrix packed in four
// complex numbers: X01 = z0, X02 = z1, X12 = z2, X00 = i Re z3, X11 = i Im z3.
template <typename T>
__device__ __forceinline__ su3<T> g_from_packed(cx<T> z0, cx<T> z1, cx<T> z2, cx<T> z3, bool exact = false) {
    su3<T> g;
    if (exact) {
        su3<T> X;
        X.e[0][0] = {T(0), z3.re};
        X.e[0][1] = z0;
        X.e[0][2] = z1;
        X.e[1][0] = {-z0.re, z0.im};
        X.e[1][1] = {T(0), z3.im};
        X.e[1][2] = z2;
        X.e[2][0] = {-z1.re, z1.im};
        X.e[2][1] = {-z2.re, z2.im};
        X.e[2][2] = {T(0), -(z3.re + z3.im)};
        g = expm_su3(X);
    } else {
        g.e[0][0] = {T(1), z3.re};
        g.e[0][1] = z0;
        g.e[0][2] = z1;
        g.e[1][0] = {-z0.re, z0.im};
        g.e[1][1] = {T(1), z3.im};
        g.e[1][2] = z2;
    }
    reunitarize_fp64(g);
    return g;
}

// ------------------------------------------------------------ link storage
// Structure-of-arrays links: entry (mu*NE + 3*row + col) of U_mu is a plane of
// ps elements, one per site. NE = 9 stores the full matrix, NE = 6 rows 1-2
// only. (Cutting the planes into tiles of 16..256 sites, so that a block's
// links form one contiguous run, measured no faster.)
// ------------------------------------------------------- per-site working arrays
// The input links U0 (4 * NE complex entries per site) and the transform H (6 per site) are kept in
// tiles of 64 consecutive sites: entry k of a tile's sites contiguous, the n entries of a tile one after
// another. A tile of U0 is a 64-site block's whole link data (36 KiB in FP64-18), so the entries a block
// reads lie in few DRAM pages (measured: 42 entries per site read at 5.9 TB/s tiled against 5.0 TB/s
// from 42 separate planes).
constexpr int kTileSites = 64;
__host__ __device__ __forceinline__ size_t tile_index(int n, int k, size_t s) {
    return ((s >> 6) * (size_t)n + (size_t)k) * kTileSites + (s & 63);
}
// The same in bytes with the entry left out (a lane's part of the address; entry k adds k * 64 elements).
template <typename T>
__device__ __forceinline__ uint32_t tile_byte_offset(int n, uint32_t s) {
    return (((s >> 6) * (uint32_t)n) * kTileSites + (s & 63)) * (uint32_t)sizeof(T);
}

template <typename T, int NE>
struct Links {
    cx<T>* p;
    size_t ps;  // elements reserved per entry (the array holds 4 * NE * ps)

    __device__ __forceinline__ size_t at(int mu, int k, size_t s) const { return tile_index(4 * NE, mu * NE + k, s); }
    __device__ __forceinline__ su3<T> load(int mu, size_t s) const {
        su3<T> u;
#pragma unroll
        for (int k = 0; k < 6; ++k) u.e[k / 3][k % 3] = p[at(mu, k, s)];
        if constexpr (NE == 9) {
#pragma unroll
            for (int k = 6; k < 9; ++k) u.e[2][k % 3] = p[at(mu, k, s)];
        } else {
            third_row(u.e[0], u.e[1], u.e[2]);
        }
        return u;
    }
    __device__ __forceinline__ void store(int mu, size_t s, const su3<T>& u) const {
#pragma unroll
        for (int k = 0; k < NE; ++k) nt_store(p + at(mu, k, s), u.e[k / 3][k % 3]);
    }
};

// --------------------------------------------------------------- geometry
struct Geom {
    int n[4];          // Nx, Ny, Nz, Nt
    int64_t vol;       // sites
    int64_t stride[4]; // 1, Nx, Nx*Ny, Nx*Ny*Nz
};

__device__ __forceinline__ void site_coords(const Geom& g, int64_t s, int c[4]) {
    uint32_t r = (uint32_t)s;
    c[0] = r % (uint32_t)g.n[0];
    r /= (uint32_t)g.n[0];
    c[1] = r % (uint32_t)g.n[1];
    r /= (uint32_t)g.n[1];
    c[2] = r % (uint32_t)g.n[2];
    c[3] = r / (uint32_t)g.n[2];
}

__device__ __forceinline__ int64_t site_back(const Geom& g, int64_t s, const int c[4], int mu) {
    return c[mu] == 0 ? s + (int64_t)(g.n[mu] - 1) * g.stride[mu] : s - g.stride[mu];
}
__device__ __forceinline__ int64_t site_fwd(const Geom& g, int64_t s, const int c[4], int mu) {
    return c[mu] == g.n[mu] - 1 ? s - (int64_t)(g.n[mu] - 1) * g.stride[mu] : s + g.stride[mu];
}

// Blocks are dealt to the 8 XCDs round-robin; give each XCD a contiguous run
// of logical tiles so that neighbouring tiles share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int xcd = b & 7, idx = b >> 3;
    return xcd < r ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

// Batch of equally shaped lattices: the buffers of configuration c sit c*cs
// bytes after those of configuration 0, and blockIdx.y picks the configuration
// (through the list of active ones when act is set). A single lattice has cs 0.
struct Batch {
    const int* act;
    size_t cs;
};

__device__ __forceinline__ size_t boff(const Batch& b) {
    if (b.cs == 0) return 0;
    const int c = b.act ? b.act[blockIdx.y] : (int)blockIdx.y;
    return (size_t)c * b.cs;
}

// Byte offset by pointer arithmetic (not through an integer), so that the compiler still sees a kernel
// argument's global address space and emits global (not flat) memory instructions.
template <typename P>
__device__ __forceinline__ P* bshift(P* p, size_t o) {
    using B = typename std::conditional<std::is_const<P>::value, const char, char>::type;
    return p ? reinterpret_cast<P*>(reinterpret_cast<B*>(p) + o) : p;
}

// ------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Deterministic block sum of two doubles; result valid in thread 0.
template <int NT>
__device__ __forceinline__ void block_sum2(double& a, double& b) {
    __shared__ double sa[NT / 64], sb[NT / 64];
    a = wave_sum(a);
    b = wave_sum(b);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) {
        sa[w] = a;
        sb[w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double ta = 0.0, tb = 0.0;
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) {
            ta += sa[i];
            tb += sb[i];
        }
        a = ta;
        b = tb;
    }
}

// ------------------------------------------------------- device control block
constexpr int kHist = 16384;

struct Ctl {
    double theta;     // quality of the current links
    double F;         // functional of the current links
    double tol;       // stop when theta < tol
    long long iters;  // updates applied
    int done;         // theta < tol reached: later kernels of the loop return at once
    int numeric;      // theta was not finite
    int pending;      // block partials of the loop kernel not yet reduced
    int guard;        // stop (rejected = 1) when an update raises theta, lowers F or is not finite
    int rejected;     // the last update was stopped by the guard
    int reserved;
    double plaquette; // mean plaquette of the links, when gf_plaquette last measured it
    double hist_theta[kHist];
    double hist_F[kHist];
};

}  // namespace gf

// Monte Carlo generator of the input ensembles: SU(3) Wilson-action heatbath
// (Cabibbo-Marinari over three SU(2) subgroups, Kennedy-Pendleton sampling),
// over-relaxation, and the multi-hit average of temporal links. The paper
// gauge-fixes thermalised configurations (Section 3) and applies multi-hit to
// the temporal links first (Section 1); it does not state the algorithms, so
// the standard ones are used:
//
//   local weight of U = U_mu(x):  exp((beta/3) Re Tr(U A)),
//   A = sum_{nu != mu} [U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag + U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu)]
//
// For a row pair (i, j) of W = U A, r = (Re(w00+w11), -Im(w01+w10), -Re(w01-w10), -Im(w00-w11))/2,
// k = |r|, V = (r0 + i r.sigma)/k; heatbath s = X V with x0 ~ sqrt(1-x0^2) exp(2 beta k x0 / 3)
// (Kennedy and Pendleton 1985) and a uniform direction; over-relaxation s = V^2. U <- s U for the
// pairs (0,1), (0,2), (1,2) in turn.
//
// Random numbers: Philox4x32-10 (Salmon, Moraes, Dror and Shaw 2011), key = the 64-bit seed, counter
// (link index 4s + mu, sweep or tag, (hit << 20) | (pair << 16) | call, purpose: 0 sweep, 1 multi-hit);
// one call gives two doubles in (0, 1] of 53 bits each. Every link's numbers depend only on its
// counter, so the result does not depend on the launch shape.
//
// The sweeps run on an even/odd structure-of-arrays copy of the links in the handle's workspace: plane
// (mu, element, parity) holds that matrix element of U_mu at the sites of that parity, site s at
// index s >> 1 (x is fastest and Nx is even, so s and s ^ 1 share an index and differ in parity).
// A wave's 64 lanes take consecutive sites of one parity, so every load and store of a link element
// is one contiguous 1 KB run. One thread per link; links of one direction and one parity share no
// staple, so each (mu, parity) half is one launch. The canonical links ([site][mu][row][col]) are
// packed before the first sweep of a call and unpacked after the last.
#pragma once

#include "gf_device.hpp"

namespace gf {

constexpr int kMcThreads = 128;
constexpr int kMcAttempts = 64;
constexpr double kMcPi = 3.14159265358979323846;

struct McGeom {
    int n[4];
    int half_x;  // Nx / 2
    long long vol;
};

__device__ __forceinline__ void philox4x32_10(unsigned c[4], unsigned k0, unsigned k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const unsigned long long p0 = 0xD2511F53ull * (unsigned long long)c[0];
        const unsigned long long p1 = 0xCD9E8D57ull * (unsigned long long)c[2];
        const unsigned hi0 = (unsigned)(p0 >> 32), lo0 = (unsigned)p0;
        const unsigned hi1 = (unsigned)(p1 >> 32), lo1 = (unsigned)p1;
        const unsigned n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

struct McKey {
    unsigned k0, k1;
    unsigned word1;   // sweep or tag
    unsigned purpose;
};

// The two uniforms of Philox call `call` for this link, pair and hit.
__device__ __forceinline__ void mc_uniforms(const McKey& key, unsigned link, int hit, int pair, int call, double& a,
                                            double& b) {
    unsigned c[4] = {link, key.word1, ((unsigned)hit << 20) | ((unsigned)pair << 16) | (unsigned)call, key.purpose};
    philox4x32_10(c, key.k0, key.k1);
    const unsigned long long ma = ((unsigned long long)c[0] << 21) | (c[1] >> 11);
    const unsigned long long mb = ((unsigned long long)c[2] << 21) | (c[3] >> 11);
    const double scale = 1.1102230246251565e-16;  // 2^-53
    a = ((double)ma + 1.0) * scale;
    b = ((double)mb + 1.0) * scale;
}

__device__ __forceinline__ su3<double> mc_load(const double2* __restrict__ links, long long s, int mu) {
    const double2* p = links + (s * 4 + mu) * 9;
    su3<double> m;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double2 v = p[k];
        m.e[k / 3][k % 3] = {v.x, v.y};
    }
    return m;
}

__device__ __forceinline__ void mc_store(double2* __restrict__ links, long long s, int mu, const su3<double>& m) {
    double2* p = links + (s * 4 + mu) * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) p[k] = {m.e[k / 3][k % 3].re, m.e[k / 3][k % 3].im};
}

// Even/odd planes: P + ((mu*9 + e)*2 + parity) * hp + (s >> 1).
struct McPlanes {
    double2* p;
    size_t hp;  // elements per plane
};

__device__ __forceinline__ int mc_parity(const int c[4]) { return (c[0] + c[1] + c[2] + c[3]) & 1; }

__device__ __forceinline__ su3<double> eo_load(const McPlanes& P, long long s, int par, int mu) {
    const double2* q = P.p + (size_t)(mu * 18 + par) * P.hp + (s >> 1);
    su3<double> m;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double2 v = q[(size_t)k * 2 * P.hp];
        m.e[k / 3][k % 3] = {v.x, v.y};
    }
    return m;
}

__device__ __forceinline__ void eo_store(const McPlanes& P, long long s, int par, int mu, const su3<double>& m) {
    double2* q = P.p + (size_t)(mu * 18 + par) * P.hp + (s >> 1);
#pragma unroll
    for (int k = 0; k < 9; ++k) q[(size_t)k * 2 * P.hp] = {m.e[k / 3][k % 3].re, m.e[k / 3][k % 3].im};
}

// a * b^dagger
__device__ __forceinline__ su3<double> mc_mul_adj(const su3<double>& a, const su3<double>& b) {
    su3<double> c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<double> s = cmulc(a.e[i][0], b.e[j][0]);
            s = cfmac(s, a.e[i][1], b.e[j][1]);
            s = cfmac(s, a.e[i][2], b.e[j][2]);
            c.e[i][j] = s;
        }
    return c;
}

// a^dagger * b
__device__ __forceinline__ su3<double> mc_adj_mul(const su3<double>& a, const su3<double>& b) {
    su3<double> c;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            cx<double> s = cmul(conj(a.e[0][i]), b.e[0][j]);
            s = cfma(s, conj(a.e[1][i]), b.e[1][j]);
            s = cfma(s, conj(a.e[2][i]), b.e[2][j]);
            c.e[i][j] = s;
        }
    return c;
}

__device__ __forceinline__ long long mc_site(const McGeom& g, const int c[4]) {
    return c[0] + (long long)g.n[0] * (c[1] + (long long)g.n[1] * (c[2] + (long long)g.n[2] * c[3]));
}

__device__ __forceinline__ long long mc_step(const McGeom& g, const int c[4], int mu, int d) {
    int e[4] = {c[0], c[1], c[2], c[3]};
    e[mu] += d;
    if (e[mu] < 0) e[mu] += g.n[mu];
    if (e[mu] >= g.n[mu]) e[mu] -= g.n[mu];
    return mc_site(g, e);
}

__device__ __forceinline__ long long mc_step2(const McGeom& g, const int c[4], int mu, int dm, int nu, int dn) {
    int e[4] = {c[0], c[1], c[2], c[3]};
    e[mu] += dm;
    e[nu] += dn;
    for (int d = 0; d < 4; ++d) {
        if (e[d] < 0) e[d] += g.n[d];
        if (e[d] >= g.n[d]) e[d] -= g.n[d];
    }
    return mc_site(g, e);
}

// Staple sum of U_mu at site coordinates c.
__device__ __forceinline__ su3<double> mc_staples(const double2* __restrict__ links, const McGeom& g, const int c[4],
                                                  int mu) {
    su3<double> a;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) a.e[i][j] = {0.0, 0.0};
    const long long s = mc_site(g, c);
    const long long s_pm = mc_step(g, c, mu, 1);
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        // U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag
        {
            const su3<double> t = mc_mul_adj(mc_load(links, s_pm, nu), mc_load(links, mc_step(g, c, nu, 1), mu));
            const su3<double> up = mc_mul_adj(t, mc_load(links, s, nu));
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) a.e[i][j] = a.e[i][j] + up.e[i][j];
        }
        // U_nu(x+mu-nu)^dag U_mu(x-nu)^dag U_nu(x-nu) = (U_mu(x-nu) U_nu(x+mu-nu))^dag U_nu(x-nu)
        {
            const long long s_mn = mc_step(g, c, nu, -1);
            const su3<double> mb = mul(mc_load(links, s_mn, mu), mc_load(links, mc_step2(g, c, mu, 1, nu, -1), nu));
            const su3<double> dn = mc_adj_mul(mb, mc_load(links, s_mn, nu));
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) a.e[i][j] = a.e[i][j] + dn.e[i][j];
        }
    }
    return a;
}

// Staple sum of U_mu at site coordinates c (parity p) from the even/odd planes; the same products in the
// same order as mc_staples. Neighbours one step away have parity 1 - p, two steps away parity p.
__device__ __forceinline__ su3<double> eo_staples(const McPlanes& P, const McGeom& g, const int c[4], int p, int mu) {
    su3<double> a;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) a.e[i][j] = {0.0, 0.0};
    const long long s = mc_site(g, c);
    const long long s_pm = mc_step(g, c, mu, 1);
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        {
            const su3<double> t = mc_mul_adj(eo_load(P, s_pm, 1 - p, nu), eo_load(P, mc_step(g, c, nu, 1), 1 - p, mu));
            const su3<double> up = mc_mul_adj(t, eo_load(P, s, p, nu));
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) a.e[i][j] = a.e[i][j] + up.e[i][j];
        }
        {
            const long long s_mn = mc_step(g, c, nu, -1);
            const su3<double> mb = mul(eo_load(P, s_mn, 1 - p, mu), eo_load(P, mc_step2(g, c, mu, 1, nu, -1), p, nu));
            const su3<double> dn = mc_adj_mul(mb, eo_load(P, s_mn, 1 - p, nu));
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) a.e[i][j] = a.e[i][j] + dn.e[i][j];
        }
    }
    return a;
}

struct Su2 {
    cx<double> m00, m01, m10, m11;
};

__device__ __forceinline__ Su2 su2_quat(double a0, double a1, double a2, double a3) {
    return {{a0, a3}, {a2, a1}, {-a2, a1}, {a0, -a3}};
}

__device__ __forceinline__ Su2 su2_mul(const Su2& a, const Su2& b) {
    return {cmul(a.m00, b.m00) + cmul(a.m01, b.m10), cmul(a.m00, b.m01) + cmul(a.m01, b.m11),
            cmul(a.m10, b.m00) + cmul(a.m11, b.m10), cmul(a.m10, b.m01) + cmul(a.m11, b.m11)};
}

__device__ __forceinline__ void su2_embed_left(const Su2& s, su3<double>& m, int i, int j) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const cx<double> ri = m.e[i][c], rj = m.e[j][c];
        m.e[i][c] = cmul(s.m00, ri) + cmul(s.m01, rj);
        m.e[j][c] = cmul(s.m10, ri) + cmul(s.m11, rj);
    }
}

// One Cabibbo-Marinari update of u with staple sum a. Returns the number of pairs left unchanged
// because every Kennedy-Pendleton attempt was rejected.
template <bool OR>
__device__ __forceinline__ int mc_cm_update(su3<double>& u, const su3<double>& a, double beta, const McKey& key,
                                            unsigned link, int hit) {
    su3<double> w = mul(u, a);
    int rejected = 0;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const int i = p == 2 ? 1 : 0, j = p == 0 ? 1 : 2;
        const cx<double> w00 = w.e[i][i], w01 = w.e[i][j], w10 = w.e[j][i], w11 = w.e[j][j];
        const double r0 = (w00.re + w11.re) / 2.0, r1 = -(w01.im + w10.im) / 2.0;
        const double r2 = -(w01.re - w10.re) / 2.0, r3 = -(w00.im - w11.im) / 2.0;
        const double k = sqrt(r0 * r0 + r1 * r1 + r2 * r2 + r3 * r3);
        if (!(k > 0.0)) continue;
        const Su2 v = su2_quat(r0 / k, r1 / k, r2 / k, r3 / k);
        Su2 s;
        if (OR) {
            s = su2_mul(v, v);
        } else {
            const double alpha = 2.0 * beta * k / 3.0;
            double x0 = 1.0;
            bool ok = false;
            for (int t = 1; t <= kMcAttempts && !ok; ++t) {
                double u1, u2, u3, u4;
                mc_uniforms(key, link, hit, p, 2 * t - 1, u1, u2);
                mc_uniforms(key, link, hit, p, 2 * t, u3, u4);
                const double cs = cos(2.0 * kMcPi * u2);
                const double delta = -(log(u1) + cs * cs * log(u3)) / alpha;
                if (u4 * u4 <= 1.0 - 0.5 * delta) {
                    x0 = 1.0 - delta;
                    ok = true;
                }
            }
            if (!ok) {
                ++rejected;
                continue;
            }
            double cu, pu;
            mc_uniforms(key, link, hit, p, 0, cu, pu);
            const double cos_t = 2.0 * cu - 1.0;
            const double sin_t = sqrt(fmax(0.0, 1.0 - cos_t * cos_t));
            const double phi = 2.0 * kMcPi * pu;
            const double rad = sqrt(fmax(0.0, 1.0 - x0 * x0));
            s = su2_mul(su2_quat(x0, rad * sin_t * cos(phi), rad * sin_t * sin(phi), rad * cos_t), v);
        }
        su2_embed_left(s, u, i, j);
        su2_embed_left(s, w, i, j);
    }
    return rejected;
}

// One (mu, parity) half-sweep: thread h updates the h-th link of direction mu among the sites of the
// given parity, in lexicographic order. Block b adds its count of rejected pair updates to rej[b]
// (plain stores: the launches of a sweep are ordered on one stream).
template <bool OR>
__global__ void __launch_bounds__(kMcThreads) k_mc_update(McPlanes P, McGeom g, int mu, int parity, double beta,
                                                          McKey key, unsigned* __restrict__ rej) {
    __shared__ unsigned red[kMcThreads];
    // Blocks visit the (x, y) planes with z in pairs inside the t loop, (z mod 2, t, z / 2), so that the t
    // neighbours were read two planes earlier and are still in the XCD's L2 (3.8 % faster per sweep at
    // 32^4 than the plain lexicographic order; groups of 4 and 8 were no better). Each link's update
    // does not depend on the order.
    long long h = (long long)blockIdx.x * kMcThreads + threadIdx.x;
    {
        const long long hpp = (long long)g.half_x * g.n[1];  // half-sites per (x, y) plane
        if (hpp % kMcThreads == 0 && g.n[2] % 2 == 0 && g.n[2] > 2) {
            const long long bpp = hpp / kMcThreads;
            const long long b = blockIdx.x, P = b / bpp, off = b - P * bpp;
            const long long z = P % 2 + 2 * (P / (2 * g.n[3]));
            const long long t = (P / 2) % g.n[3];
            h = ((z + (long long)g.n[2] * t) * bpp + off) * kMcThreads + threadIdx.x;
        }
    }
    unsigned rj = 0;
    if (h < g.vol / 2) {
        const long long row = h / g.half_x;
        int c[4];
        c[1] = (int)(row % g.n[1]);
        c[2] = (int)((row / g.n[1]) % g.n[2]);
        c[3] = (int)(row / ((long long)g.n[1] * g.n[2]));
        c[0] = 2 * (int)(h - row * g.half_x) + ((c[1] + c[2] + c[3] + parity) & 1);
        const long long s = mc_site(g, c);
        const su3<double> a = eo_staples(P, g, c, parity, mu);
        su3<double> u = eo_load(P, s, parity, mu);
        rj = (unsigned)mc_cm_update<OR>(u, a, beta, key, (unsigned)(s * 4 + mu), 0);
        eo_store(P, s, parity, mu, u);
    }
    if (OR) return;
    red[threadIdx.x] = rj;
    __syncthreads();
    for (int w = kMcThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0]) rej[blockIdx.x] += red[0];
}

// Canonical links <-> even/odd planes, one thread per site.
__global__ void __launch_bounds__(256) k_mc_pack(const double2* __restrict__ links, McPlanes P, McGeom g) {
    const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
    if (s >= g.vol) return;
    int c[4];
    long long r = s;
    for (int d = 0; d < 4; ++d) {
        c[d] = (int)(r % g.n[d]);
        r /= g.n[d];
    }
    const int par = mc_parity(c);
    for (int mu = 0; mu < 4; ++mu) eo_store(P, s, par, mu, mc_load(links, s, mu));
}

__global__ void __launch_bounds__(256) k_mc_unpack(McPlanes P, McGeom g, double2* __restrict__ links) {
    const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
    if (s >= g.vol) return;
    int c[4];
    long long r = s;
    for (int d = 0; d < 4; ++d) {
        c[d] = (int)(r % g.n[d]);
        r /= g.n[d];
    }
    const int par = mc_parity(c);
    for (int mu = 0; mu < 4; ++mu) mc_store(links, s, mu, eo_load(P, s, par, mu));
}

// Every link reunitarised in the planes: thread per (site of one parity index, parity, mu).
__global__ void __launch_bounds__(256) k_mc_reunit(McPlanes P, long long half) {
    const long long l = (long long)blockIdx.x * 256 + threadIdx.x;  // l = (mu * 2 + parity) * half + h
    if (l >= 8 * half) return;
    const long long h = l % half;
    const int mp = (int)(l / half), mu = mp >> 1, par = mp & 1;
    double2* q = P.p + (size_t)(mu * 18 + par) * P.hp + h;
    su3<double> m;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double2 v = q[(size_t)k * 2 * P.hp];
        m.e[k / 3][k % 3] = {v.x, v.y};
    }
    reunitarize(m);
#pragma unroll
    for (int k = 0; k < 9; ++k) q[(size_t)k * 2 * P.hp] = {m.e[k / 3][k % 3].re, m.e[k / 3][k % 3].im};
}

__global__ void __launch_bounds__(256) k_mc_zero(unsigned* __restrict__ p, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Sum of n counters into *out (one block, fixed order).
__global__ void __launch_bounds__(256) k_mc_count(const unsigned* __restrict__ p, int n,
                                                  unsigned long long* __restrict__ out) {
    __shared__ unsigned long long red[256];
    unsigned long long v = 0;
    for (int i = threadIdx.x; i < n; i += 256) v += p[i];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// Multi-hit average of every temporal link, out as complex double [site][row][col].
__global__ void __launch_bounds__(kMcThreads) k_mc_multihit(const double2* __restrict__ links, McGeom g,
                                                            double beta, McKey key, int nhits,
                                                            double2* __restrict__ out) {
    const long long s = (long long)blockIdx.x * kMcThreads + threadIdx.x;
    if (s >= g.vol) return;
    int c[4];
    long long r = s;
    for (int d = 0; d < 4; ++d) {
        c[d] = (int)(r % g.n[d]);
        r /= g.n[d];
    }
    const su3<double> a = mc_staples(links, g, c, 3);
    su3<double> u = mc_load(links, s, 3);
    su3<double> acc;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) acc.e[i][j] = {0.0, 0.0};
    for (int h = 0; h < nhits; ++h) {
        (void)mc_cm_update<false>(u, a, beta, key, (unsigned)(s * 4 + 3), h);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) acc.e[i][j] = acc.e[i][j] + u.e[i][j];
    }
    double2* p = out + s * 9;
#pragma unroll
    for (int k = 0; k < 9; ++k) p[k] = {acc.e[k / 3][k % 3].re / nhits, acc.e[k / 3][k % 3].im / nhits};
}

// Plaquette partials: block b sums Re Tr of the six plaquettes at each of its sites (fixed order).
__global__ void __launch_bounds__(256) k_mc_plaquette(const double2* __restrict__ links, McGeom g,
                                                      double* __restrict__ part) {
    __shared__ double red[256];
    const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
    double v = 0.0;
    if (s < g.vol) {
        int c[4];
        long long r = s;
        for (int d = 0; d < 4; ++d) {
            c[d] = (int)(r % g.n[d]);
            r /= g.n[d];
        }
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                const su3<double> t = mul(mc_load(links, s, mu), mc_load(links, mc_step(g, c, mu, 1), nu));
                const su3<double> q = mc_mul_adj(mc_mul_adj(t, mc_load(links, mc_step(g, c, nu, 1), mu)),
                                                 mc_load(links, s, nu));
                v += q.e[0][0].re + q.e[1][1].re + q.e[2][2].re;
            }
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_mc_plaquette_sum(const double* __restrict__ part, int n, double scale,
                                                          double* __restrict__ out) {
    __shared__ double red[256];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) v += part[i];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

}  // namespace gf

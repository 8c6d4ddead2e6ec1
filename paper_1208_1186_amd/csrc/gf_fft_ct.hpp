// FFT pass kernels specialised at compile time for the plane shapes of the
// standard workloads (x-y planes 8^2 .. 48^2, z-t planes of the 8^4, 12^4,
// 16^4, 24^3x8, 32^3x4, 48^3x8, 32^4 and 32^3x64 lattices). They compute
// exactly what the runtime-shaped kernels in gf_kernels.hpp compute; other
// shapes use those.
#pragma once

#include "gf_kernels.hpp"

namespace gf {

constexpr int ct_threads(int elems, int ept) {
    const int t = (elems + ept - 1) / ept;
    const int r = (t + 63) / 64 * 64;
    return r < 64 ? 64 : (r > 1024 ? 1024 : r);
}

// (x, y) pass over G single-field planes per block, src -> dst.
template <typename T, int NX, int NY, int G, bool INV>
__global__ void __launch_bounds__(ct_threads(G * NX * NY, 8))
    k_fft_xy_ct(const cx<T>* src, cx<T>* dst, size_t zps, int nzt, const cx<T>* __restrict__ twgx,
                const cx<T>* __restrict__ twgy, Ctl* ctl, int force, const double2* __restrict__ part, int npart,
                double inv3v, double inv12v, Batch bt) {
    constexpr int RS = NX + 1, E = G * NX * NY, NT = ct_threads(E, 8);
    {
        const size_t bo = boff(bt);
        src = bshift(src, bo);
        dst = bshift(dst, bo);
        twgx = bshift(twgx, bo);
        twgy = bshift(twgy, bo);
        ctl = bshift(ctl, bo);
        part = bshift(part, bo);
    }
    if (part != nullptr && blockIdx.x == 0 && ctl->pending) {
        reduce_partials(part, npart, inv3v, inv12v, ctl, 1);
        __syncthreads();
    }
    if (!force && ctl->done) return;
    __shared__ cx<T> twx[NX], twy[NY], buf[G * NY * RS];
    for (int i = threadIdx.x; i < NX; i += NT) twx[i] = twgx[i];
    for (int i = threadIdx.x; i < NY; i += NT) twy[i] = twgy[i];
    const int q0 = xcd_remap(blockIdx.x, gridDim.x) * G;
    const int f = q0 / nzt, zt0 = q0 - f * nzt;
    const size_t off = (size_t)f * zps + (size_t)zt0 * NX * NY;
    const cx<T>* gs = src + off;
    cx<T>* gd = dst + off;
#pragma unroll
    for (int e0 = 0; e0 < E; e0 += NT) {
        const int e = e0 + threadIdx.x;
        if (E % NT == 0 || e < E) buf[(e / NX) * RS + e % NX] = gs[e];
    }
    __syncthreads();
    fft_rows_ct<NX, 0, 1, Rows<G * NY, 1, G * NY, RS, 0>, NT, T, INV>(buf, twx);
    fft_rows_ct<NY, 0, 1, Rows<G * NX, RS, NX, 1, NY * RS>, NT, T, INV>(buf, twy);
#pragma unroll
    for (int e0 = 0; e0 < E; e0 += NT) {
        const int e = e0 + threadIdx.x;
        if (E % NT == 0 || e < E) gd[e] = buf[(e / NX) * RS + e % NX];
    }
}

// (z, t) pass with the filter, BX x columns per block, in place.
template <typename T, int NZ, int NTT, int BX>
__global__ void __launch_bounds__(ct_threads(BX * NZ * NTT, 8))
    k_fft_zt_ct(cx<T>* __restrict__ Z, size_t zps, int nx, int ny, const cx<T>* __restrict__ twgz,
                const cx<T>* __restrict__ twgt, const T* __restrict__ sin2, T coef, int no_fa,
                const Ctl* __restrict__ ctl, int force, const T* __restrict__ mtab, TupleGeom tg,
                cx<T>* __restrict__ spec, Batch bt) {
    // LDS row pitch NZ*BX + BX: along a z row the lanes step through (x, t) as xo + TSP*t, so with
    // TSP = BX (mod the number of element slots per LDS cycle) consecutive lanes land in consecutive
    // slots; a pitch of NZ*BX + 1 put the lanes of neighbouring t rows on the same slots when BX > 1
    // (measured: the pass 2-3 us faster at 32^4 and 48^3x8).
    constexpr int TSP = NZ * BX + BX, E = BX * NZ * NTT, NT = ct_threads(E, 8);
    {
        const size_t bo = boff(bt);
        Z = bshift(Z, bo);
        twgz = bshift(twgz, bo);
        twgt = bshift(twgt, bo);
        sin2 = bshift(sin2, bo);
        ctl = bshift(ctl, bo);
    }
    if (!force && ctl->done) return;
    __shared__ cx<T> twz[NZ], twt[NTT], buf[NTT * TSP];
    for (int i = threadIdx.x; i < NZ; i += NT) twz[i] = twgz[i];
    for (int i = threadIdx.x; i < NTT; i += NT) twt[i] = twgt[i];
    const int nxb = nx / BX;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int xb = blk % nxb;
    const int rest = blk / nxb;
    const int y = rest % ny, f = rest / ny;
    const int x0 = xb * BX;
    cx<T>* gp = Z + (size_t)f * zps + x0 + (size_t)nx * y;
    const size_t pstep = (size_t)nx * ny;
#pragma unroll
    for (int e0 = 0; e0 < E; e0 += NT) {
        const int e = e0 + threadIdx.x;
        if (E % NT == 0 || e < E) {
            const int xo = e % BX, zt = e / BX;
            buf[(zt / NZ) * TSP + (zt % NZ) * BX + xo] = gp[xo + zt * pstep];
        }
    }
    __syncthreads();
    fft_rows_ct<NZ, 0, 1, Rows<NTT * BX, BX, BX, 1, TSP>, NT, T, false>(buf, twz);
    fft_rows_ct<NTT, 0, 1, Rows<NZ * BX, TSP, NZ * BX, 1, 0>, NT, T, false>(buf, twt);
    const T* sx = sin2;
    const T* sy = sin2 + nx;
    const T* sz = sy + ny;
    const T* st = sz + NZ;
    const T sxy = sy[y];
#pragma unroll
    for (int e0 = 0; e0 < E; e0 += NT) {
        const int e = e0 + threadIdx.x;
        if (E % NT == 0 || e < E) {
            const int xo = e % BX, zt = e / BX;
            const int z = zt % NZ, t = zt / NZ;
            const int li = t * TSP + z * BX + xo;
            if (spec) spec[xo + zt * pstep + (gp - Z)] = buf[li];
            T mult;
            if (mtab) {
                mult = mtab[tuple_index(tg, x0 + xo, y, z, t)];
            } else {
                const T p2 = sx[x0 + xo] + sxy + sz[z] + st[t];
                mult = p2 > T(0) ? (no_fa ? coef : coef / p2) : T(0);
            }
            buf[li] = cscale(buf[li], mult);
        }
    }
    __syncthreads();
    fft_rows_ct<NTT, 0, 1, Rows<NZ * BX, TSP, NZ * BX, 1, 0>, NT, T, true>(buf, twt);
    fft_rows_ct<NZ, 0, 1, Rows<NTT * BX, BX, BX, 1, TSP>, NT, T, true>(buf, twz);
#pragma unroll
    for (int e0 = 0; e0 < E; e0 += NT) {
        const int e = e0 + threadIdx.x;
        if (E % NT == 0 || e < E) {
            const int xo = e % BX, zt = e / BX;
            gp[xo + zt * pstep] = buf[(zt / NZ) * TSP + (zt % NZ) * BX + xo];
        }
    }
}

// Inverse (x, y) pass of the four fields of one (z, t) plane, then g and the update of the stored
// transform, Hout = reunitarize(g Hin) (rows 1-2); with Hin null, g itself goes to Hout.
constexpr int gauge_ept(int nx, int ny) { return 4 * nx * ny <= 8 * 1024 ? 8 : 16; }

template <typename T, int NX, int NY>
__global__ void __launch_bounds__(ct_threads(4 * NX * NY, gauge_ept(NX, NY)))
    k_fft_xy_gauge_ct(const cx<T>* __restrict__ Q, size_t zps, const cx<T>* __restrict__ Hin,
                      cx<T>* __restrict__ Hout, const cx<T>* __restrict__ twgx,
                      const cx<T>* __restrict__ twgy, const Ctl* __restrict__ ctl, int force, Batch bt, int exact) {
    constexpr int RS = NX + 1, P = NX * NY, PL = NY * RS, E = 4 * P;
    constexpr int NT = ct_threads(E, gauge_ept(NX, NY));
    {
        const size_t bo = boff(bt);
        Q = bshift(Q, bo);
        Hin = bshift(Hin, bo);
        Hout = bshift(Hout, bo);
        twgx = bshift(twgx, bo);
        twgy = bshift(twgy, bo);
        ctl = bshift(ctl, bo);
    }
    if (!force && ctl->done) return;
    extern __shared__ __align__(16) unsigned char smem[];
    cx<T>* twx = reinterpret_cast<cx<T>*>(smem);
    cx<T>* twy = twx + NX;
    cx<T>* buf = twy + NY;
    for (int i = threadIdx.x; i < NX; i += NT) twx[i] = twgx[i];
    for (int i = threadIdx.x; i < NY; i += NT) twy[i] = twgy[i];
    const size_t base = (size_t)xcd_remap(blockIdx.x, gridDim.x) * P;
#pragma unroll
    for (int e0 = 0; e0 < E; e0 += NT) {
        const int e = e0 + threadIdx.x;
        if (E % NT == 0 || e < E) {
            const int f = e / P, r = e % P;
            buf[f * PL + (r / NX) * RS + r % NX] = Q[(size_t)f * zps + base + r];
        }
    }
    __syncthreads();
    fft_rows_ct<NX, 0, 1, Rows<4 * NY, 1, 4 * NY, RS, 0>, NT, T, true>(buf, twx);
    fft_rows_ct<NY, 0, 1, Rows<4 * NX, RS, NX, 1, PL>, NT, T, true>(buf, twy);
#pragma unroll
    for (int r0 = 0; r0 < P; r0 += NT) {
        const int r = r0 + threadIdx.x;
        if (P % NT == 0 || r < P) {
            const int li = (r / NX) * RS + r % NX;
            su3<T> g = g_from_packed(buf[li], buf[PL + li], buf[2 * PL + li], buf[3 * PL + li], exact != 0);
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
}

constexpr size_t gauge_ct_lds(int nx, int ny, size_t csz) { return (size_t)(nx + ny + 4 * ny * (nx + 1)) * csz; }

}  // namespace gf

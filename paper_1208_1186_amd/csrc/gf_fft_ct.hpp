// FFT pass kernels specialised at compile time for the plane shapes of the
// standard workloads (x-y planes 8^2 .. 48^2, z-t planes of the 8^4, 12^4,
// 16^4, 24^3x8, 32^3x4, 48^3x8, 32^4 and 32^3x64 lattices). They compute the
// same transforms as the runtime-shaped kernels in gf_kernels.hpp (which
// other shapes use), with some stages reading or writing memory directly; the
// inverse t transform takes its radices in the reverse order and the inverse
// (x, y) pass transforms y first, so the two families agree to rounding, and
// all tilings of one family bitwise.
#pragma once

#include "gf_kernels.hpp"

namespace gf {

constexpr int ct_threads(int elems, int ept) {
    const int t = (elems + ept - 1) / ept;
    const int r = (t + 63) / 64 * 64;
    return r < 64 ? 64 : (r > 1024 ? 1024 : r);
}

// Row b of the y transforms of a block's planes is column b % NX of plane b / NX; the last y
// stage writes element e (its y) straight to memory, a run of NX consecutive sites per plane row.
template <typename T, int NX, int NY>
struct XyOut {
    cx<T>* gd;
    static constexpr bool lds_in = false, lds_out = false;
    __device__ __forceinline__ void st(int b, int e, cx<T> v) const { gd[(b / NX) * (NX * NY) + e * NX + b % NX] = v; }
};

// (x, y) pass over G single-field planes per block, src -> dst (one more block when part is set).
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
    // With part set, block 0 (dispatched first) only reduces the loop kernel's pending partials and
    // the other blocks transform: a block that did both ended last on small tilings.
    const int red = part != nullptr ? 1 : 0;
    if (red && blockIdx.x == 0) {
        if (ctl->pending) reduce_partials(part, npart, inv3v, inv12v, ctl, 1);
        return;
    }
    if (!force && ctl->done) return;
    __shared__ cx<T> twx[NX], twy[NY], buf[G * NY * RS];
    for (int i = threadIdx.x; i < NX; i += NT) twx[i] = twgx[i];
    for (int i = threadIdx.x; i < NY; i += NT) twy[i] = twgy[i];
    const int q0 = xcd_remap(blockIdx.x - red, gridDim.x - red) * G;
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
    using RY = Rows<G * NX, RS, NX, 1, NY * RS>;
    fft_rows_io<NY, 0, 1, RY, NT, T, INV>(buf, twy, LdsIo<RY, T>{buf}, XyOut<T, NX, NY>{gd}, threadIdx.x);
}

// Global side of the (z, t) pass: row b of the z transforms is the column (x0 + b % BX, y) at
// t = b / BX, element e its z; the block's first z stage reads from here and its last inverse z
// stage writes back here.
template <typename T, int NZ, int BX>
struct ZtGlobal {
    cx<T>* gp;
    int pstep;
    static constexpr bool lds_in = false, lds_out = false;
    __device__ __forceinline__ int at(int b, int e) const { return b % BX + (e + NZ * (b / BX)) * pstep; }
    __device__ __forceinline__ cx<T> ld(int b, int e) const { return gp[at(b, e)]; }
    __device__ __forceinline__ void st(int b, int e, cx<T> v) const { gp[at(b, e)] = v; }
};

// The filter on the spectrum at (x0 + xo, y, z, t) (row b = z*BX + xo of the t transforms,
// element e = t), which it records first when asked. The sin^2 tables are in LDS (filled before
// the block's first barrier, read only after it).
template <typename T, int NZ, int BX>
struct ZtFilter {
    cx<T>* spec;  // spectrum record at the block's first column, or null
    const T *sx, *sy, *sz, *stt;  // sin^2 tables along x (from x0), y, z and t
    const T* mtab;
    TupleGeom tg;
    T coef;
    int no_fa, x0, y, pstep;
    __device__ __forceinline__ cx<T> apply(int b, int e, cx<T> v) const {
        const int xo = b % BX, z = b / BX, t = e;
        if (spec) spec[xo + (z + NZ * t) * pstep] = v;
        T mult;
        if (mtab) {
            mult = mtab[tuple_index(tg, x0 + xo, y, z, t)];
        } else {
            const T p2 = sx[xo] + sy[y] + sz[z] + stt[t];
            mult = p2 > T(0) ? (no_fa ? coef : coef / p2) : T(0);
        }
        return cscale(v, mult);
    }
};

// Largest x or y extent the compile-time (z, t) passes take (their sin^2 tables sit in LDS).
constexpr int kZtMaxXY = 64;

// (z, t) pass with the filter, BX x columns per block, in place. The first z stage reads the
// columns from memory and the last inverse z stage writes them back; the filter and the first
// inverse t stage work on the last forward t stage's registers.
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
    using RZ = Rows<NTT * BX, BX, BX, 1, TSP>;
    using RT = Rows<NZ * BX, TSP, NZ * BX, 1, 0>;
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
    __shared__ T s2[2 * kZtMaxXY + NZ + NTT];  // sin^2 along x, y, z, t
    for (int i = threadIdx.x; i < NZ; i += NT) twz[i] = twgz[i];
    for (int i = threadIdx.x; i < NTT; i += NT) twt[i] = twgt[i];
    for (int i = threadIdx.x; i < nx; i += NT) s2[i] = sin2[i];
    for (int i = threadIdx.x; i < ny; i += NT) s2[kZtMaxXY + i] = sin2[nx + i];
    for (int i = threadIdx.x; i < NZ + NTT; i += NT) s2[2 * kZtMaxXY + i] = sin2[nx + ny + i];
    const int nxb = nx / BX;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int xb = blk % nxb;
    const int rest = blk / nxb;
    const int y = rest % ny, f = rest / ny;
    const int x0 = xb * BX;
    const size_t goff = (size_t)f * zps + x0 + (size_t)nx * y;
    const int pstep = nx * ny;
    const int tid = threadIdx.x;
    const ZtGlobal<T, NZ, BX> col{Z + goff, pstep};
    const LdsIo<RZ, T> lds_z{buf};
    const ZtFilter<T, NZ, BX> filt{spec ? spec + goff : nullptr, s2 + x0, s2 + kZtMaxXY, s2 + 2 * kZtMaxXY,
                                        s2 + 2 * kZtMaxXY + NZ, mtab, tg, coef, no_fa,
                                        x0, y, pstep};
    fft_rows_io<NZ, 0, 1, RZ, NT, T, false>(buf, twz, col, lds_z, tid);
    fft_rows_map_inverse<NTT, RT, NT, T>(buf, twt, filt, tid);
    fft_rows_io<NZ, 0, 1, RZ, NT, T, true>(buf, twz, lds_z, col, tid);
}

// Row b of the y transforms of one (z, t) plane's four fields is column b % NX of field b / NX;
// the first y stage reads element e (its y) straight from memory, runs of NX consecutive sites.
template <typename T, int NX>
struct PlaneIn {
    const cx<T>* q;  // the plane's first site in field 0
    size_t zps;      // field stride
    static constexpr bool lds_in = false, lds_out = false;
    __device__ __forceinline__ cx<T> ld(int b, int e) const { return q[(size_t)(b / NX) * zps + e * NX + b % NX]; }
};

// Inverse (x, y) pass of the four fields of one (z, t) plane (y transforms first, read from
// memory), then g and the update of the stored transform, Hout = reunitarize(g Hin) (rows 1-2);
// with Hin null, g itself goes to Hout. Elements per thread: 8 up to 32 x 32 planes, 9 on 48 x 48
// (1024 threads; with 16 the few blocks of such lattices, 384 at 48^3 x 8, ran 9 waves each and the
// pass took 34 us in float against 26, 59 in double against 54).
constexpr int gauge_ept(int nx, int ny) { return 4 * nx * ny <= 8 * 1024 ? 8 : 4 * nx * ny <= 9 * 1024 ? 9 : 16; }

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
    using RY = Rows<4 * NX, RS, NX, 1, PL>;
    fft_rows_io<NY, 0, 1, RY, NT, T, true>(buf, twy, PlaneIn<T, NX>{Q + base, zps}, LdsIo<RY, T>{buf},
                                           threadIdx.x);
    fft_rows_ct<NX, 0, 1, Rows<4 * NY, 1, 4 * NY, RS, 0>, NT, T, true>(buf, twx);
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

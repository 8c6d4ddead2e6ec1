// (z, t) pass with whole transforms held in registers: each thread owns one line of a (z, t) plane,
// transforms it in its registers (no LDS traffic inside a transform), and the planes change hands
// through LDS only between the z and the t transforms: two exchanges and two barriers per pass, against
// one exchange and two barriers per radix stage in the LDS Stockham passes.
#pragma once

#include "gf_fft_ct.hpp"

namespace gf {

// Index j of a length-N (power of two) transform with its bits reversed.
template <int N>
__host__ __device__ constexpr int bitrev(int j) {
    int r = 0;
    for (int m = N >> 1, b = 1; m > 0; m >>= 1, b <<= 1)
        if (j & b) r |= m;
    return r;
}

// In-register radix-2 transforms of x[0..N-1] in place (N a power of two; every index is known at compile
// time, so the array stays in registers). fft_dif: natural order in, bit-reversed order out (x[j] holds
// mode bitrev(j)); fft_dit: bit-reversed order in, natural order out. The twiddle W_len^k is
// tw[k * NTAB / len], tw the table of the NTAB-th roots exp(-2 pi i k / NTAB) (conjugated for the
// inverse). Forward and inverse are unnormalised, as in the LDS passes.
template <typename T, bool INV>
__device__ __forceinline__ cx<T> twiddle(const cx<T>* __restrict__ tw, int i) {
    cx<T> w = tw[i];
    if (INV) w.im = -w.im;
    return w;
}

template <typename T, int N, int NTAB, bool INV>
__device__ __forceinline__ void fft_dif(cx<T>* x, const cx<T>* __restrict__ tw) {
#pragma unroll
    for (int len = N; len >= 2; len >>= 1) {
#pragma unroll
        for (int i = 0; i < N; i += len) {
#pragma unroll
            for (int k = 0; k < len / 2; ++k) {
                const cx<T> a = x[i + k], b = x[i + k + len / 2];
                x[i + k] = a + b;
                x[i + k + len / 2] = k == 0 ? a - b : cmul(a - b, twiddle<T, INV>(tw, k * (NTAB / len)));
            }
        }
    }
}

template <typename T, int N, int NTAB, bool INV>
__device__ __forceinline__ void fft_dit(cx<T>* x, const cx<T>* __restrict__ tw) {
#pragma unroll
    for (int len = 2; len <= N; len <<= 1) {
#pragma unroll
        for (int i = 0; i < N; i += len) {
#pragma unroll
            for (int k = 0; k < len / 2; ++k) {
                const cx<T> a = x[i + k];
                const cx<T> b = k == 0 ? x[i + k + len / 2] : cmul(x[i + k + len / 2], twiddle<T, INV>(tw, k * (NTAB / len)));
                x[i + k] = a + b;
                x[i + k + len / 2] = a - b;
            }
        }
    }
}

// (z, t) pass with the filter, BX consecutive x columns at one y of one field per block, in place
// (NZ, NTT powers of two up to 32). Thread (xo, t) loads the z line, transforms it and writes it to LDS
// (element (xo, z, t) at t*TP + z*BX + xo; the pitch TP = NZ*BX + BX puts the 16 lanes of one 256-byte
// LDS pass on distinct slots); thread (xo, z) then transforms the t line, multiplies every mode by coef /
// p^2(p) (zero mode -> 0; coef alone when no_fa; the learned table when mtab is set) and transforms
// back; thread (xo, t) finally takes the inverse z transform and stores the line.
template <typename T, int NZ, int NTT, int BX>
__global__ void __launch_bounds__(BX*(NZ > NTT ? NZ : NTT))
    k_fft_zt_reg(cx<T>* __restrict__ Z, size_t zps, int nx, int ny, const cx<T>* __restrict__ twgz,
                 const cx<T>* __restrict__ twgt, const T* __restrict__ sin2, T coef, int no_fa,
                 const Ctl* __restrict__ ctl, int force, const T* __restrict__ mtab, TupleGeom tg,
                 cx<T>* __restrict__ spec, Batch bt) {
    constexpr int TP = NZ * BX + BX;
    {
        const size_t bo = boff(bt);
        Z = bshift(Z, bo);
        twgz = bshift(twgz, bo);
        twgt = bshift(twgt, bo);
        sin2 = bshift(sin2, bo);
        ctl = bshift(ctl, bo);
    }
    if (!force && ctl->done) return;
    __shared__ cx<T> buf[NTT * TP];
    const int nxb = nx / BX;
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int xb = blk % nxb;
    const int rest = blk / nxb;
    const int y = rest % ny, f = rest / ny;
    const int x0 = xb * BX;
    cx<T>* gp = Z + (size_t)f * zps + x0 + (size_t)nx * y;
    const size_t pstep = (size_t)nx * ny;
    const int tid = threadIdx.x;
    const int xo = tid % BX, line = tid / BX;
    if (line < NTT) {  // z lines: line = t; forward z transform, modes to LDS in natural order
        cx<T> v[NZ];
#pragma unroll
        for (int z = 0; z < NZ; ++z) v[z] = gp[xo + (size_t)(z + NZ * line) * pstep];
        fft_dif<T, NZ, NZ, false>(v, twgz);
#pragma unroll
        for (int j = 0; j < NZ; ++j) buf[line * TP + bitrev<NZ>(j) * BX + xo] = v[j];
    }
    __syncthreads();
    if (line < NZ) {  // t lines: line = z (mode); forward t transform, filter, inverse t transform
        const int z = line;
        cx<T> v[NTT];
#pragma unroll
        for (int t = 0; t < NTT; ++t) v[t] = buf[t * TP + z * BX + xo];
        fft_dif<T, NTT, NTT, false>(v, twgt);  // v[j] holds t mode bitrev(j)
        const T* sx = sin2;
        const T* sy = sin2 + nx;
        const T* sz = sy + ny;
        const T* st = sz + NZ;
        const T pxyz = sx[x0 + xo] + sy[y] + sz[z];
#pragma unroll
        for (int j = 0; j < NTT; ++j) {
            const int t = bitrev<NTT>(j);
            if (spec) spec[(gp - Z) + xo + (size_t)(z + NZ * t) * pstep] = v[j];
            T mult;
            if (mtab) {
                mult = mtab[tuple_index(tg, x0 + xo, y, z, t)];
            } else {
                const T p2 = pxyz + st[t];
                mult = p2 > T(0) ? (no_fa ? coef : coef / p2) : T(0);
            }
            v[j] = cscale(v[j], mult);
        }
        fft_dit<T, NTT, NTT, true>(v, twgt);  // back in natural t order
#pragma unroll
        for (int t = 0; t < NTT; ++t) buf[t * TP + z * BX + xo] = v[t];
    }
    __syncthreads();
    if (line < NTT) {  // inverse z transform (modes read in bit-reversed order), store
        cx<T> v[NZ];
#pragma unroll
        for (int j = 0; j < NZ; ++j) v[j] = buf[line * TP + bitrev<NZ>(j) * BX + xo];
        fft_dit<T, NZ, NZ, true>(v, twgz);
#pragma unroll
        for (int z = 0; z < NZ; ++z) gp[xo + (size_t)(z + NZ * line) * pstep] = v[z];
    }
}

}  // namespace gf

// Mixed-radix (2, 3, 4, 8) Stockham FFT stages over data resident in LDS.
//
// A length-N transform (N = 2^a 3^b) is a sequence of radix-R stages. With
// p the product of the radices already applied and m = N/R, butterfly i of a
// row reads x[i + j*m] (j < R), multiplies input j by W_{pR}^{j*(i mod p)},
// takes an R-point DFT and writes output j to y[(i - i mod p)*R + i mod p + j*p]
// (the first stage, p = 1, has no twiddles: they are all 1).
// The result comes out in natural order (self-sorting). A stage works in
// place: every thread first loads all its butterflies into registers, the
// block synchronises, then every thread writes its outputs.
//
// Forward transforms use W_N = exp(-2 pi i / N) and are unnormalised; inverse
// transforms use the conjugate roots and are unnormalised too.
#pragma once

#include "gf_device.hpp"

namespace gf {

struct FftPlan {
    int n;        // transform length
    int nst;      // number of stages
    int rad[6];   // radix of each stage
};

template <typename T, bool INV>
__device__ __forceinline__ cx<T> mul_mi(cx<T> a) {  // a * (-i) forward, a * (+i) inverse
    return INV ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re};
}

template <int R, typename T, bool INV>
__device__ __forceinline__ void dft_small(cx<T>* v) {
    if constexpr (R == 2) {
        cx<T> a = v[0], b = v[1];
        v[0] = a + b;
        v[1] = a - b;
    } else if constexpr (R == 3) {
        // X1,2 = a - (b+c)/2 -/+ i (sqrt(3)/2)(b - c) (forward)
        const T s3 = T(0.86602540378443864676372317075294);
        cx<T> a = v[0], t1 = v[1] + v[2], t2 = v[1] - v[2];
        cx<T> mid = {a.re - T(0.5) * t1.re, a.im - T(0.5) * t1.im};
        cx<T> rot = {-s3 * t2.im, s3 * t2.re};  // i * s3 * t2
        v[0] = a + t1;
        if (INV) {
            v[1] = mid + rot;
            v[2] = mid - rot;
        } else {
            v[1] = mid - rot;
            v[2] = mid + rot;
        }
    } else if constexpr (R == 4) {
        cx<T> s02 = v[0] + v[2], d02 = v[0] - v[2];
        cx<T> s13 = v[1] + v[3], d13 = mul_mi<T, INV>(v[1] - v[3]);
        v[0] = s02 + s13;
        v[2] = s02 - s13;
        v[1] = d02 + d13;
        v[3] = d02 - d13;
    } else if constexpr (R == 8) {
        const T h = T(0.70710678118654752440084436210485);
        cx<T> e[4] = {v[0], v[2], v[4], v[6]};
        cx<T> o[4] = {v[1], v[3], v[5], v[7]};
        dft_small<4, T, INV>(e);
        dft_small<4, T, INV>(o);
        // W8^1 = (1 -/+ i)/sqrt2, W8^2 = -/+ i, W8^3 = (-1 -/+ i)/sqrt2
        cx<T> o1 = INV ? cx<T>{h * (o[1].re - o[1].im), h * (o[1].re + o[1].im)}
                       : cx<T>{h * (o[1].re + o[1].im), h * (o[1].im - o[1].re)};
        cx<T> o2 = mul_mi<T, INV>(o[2]);
        cx<T> o3 = INV ? cx<T>{-h * (o[3].re + o[3].im), h * (o[3].re - o[3].im)}
                       : cx<T>{h * (o[3].im - o[3].re), -h * (o[3].re + o[3].im)};
        v[0] = e[0] + o[0];
        v[4] = e[0] - o[0];
        v[1] = e[1] + o1;
        v[5] = e[1] - o1;
        v[2] = e[2] + o2;
        v[6] = e[2] - o2;
        v[3] = e[3] + o3;
        v[7] = e[3] - o3;
    }
}

// One radix-R stage over nrows rows of length N in LDS. Row b starts at
// (b % n0)*s0 + (b / n0)*s1 and its elements are es apart. Consecutive
// threads take consecutive rows. EPT bounds the elements each thread holds.
template <int R, int EPT, typename T, bool INV>
__device__ __forceinline__ void fft_stage(cx<T>* buf, const cx<T>* tw, int N, int p, int es, int nrows,
                                          int n0, int s0, int s1) {
    constexpr int IMAX = (EPT + R - 1) / R;
    const int m = N / R;
    const int items = nrows * m;
    const int nt = blockDim.x;
    const int twstep = N / (p * R);
    cx<T> v[IMAX][R];
    int obase[IMAX];
#pragma unroll
    for (int it = 0; it < IMAX; ++it) {
        const int w = threadIdx.x + it * nt;
        if (w < items) {
            const int b = w % nrows, i = w / nrows;
            const int base = (b % n0) * s0 + (b / n0) * s1;
            const int k = i % p;
#pragma unroll
            for (int j = 0; j < R; ++j) v[it][j] = buf[base + (i + j * m) * es];
            obase[it] = base + ((i - k) * R + k) * es;
            if (p > 1) {  // the first stage's twiddles are all 1
#pragma unroll
                for (int j = 1; j < R; ++j) {
                    cx<T> t = tw[j * k * twstep];
                    if (INV) t.im = -t.im;
                    v[it][j] = cmul(v[it][j], t);
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IMAX; ++it) {
        const int w = threadIdx.x + it * nt;
        if (w < items) {
            dft_small<R, T, INV>(v[it]);
#pragma unroll
            for (int j = 0; j < R; ++j) buf[obase[it] + j * p * es] = v[it][j];
        }
    }
    __syncthreads();
}

template <int EPT, typename T, bool INV>
__device__ __forceinline__ void fft_rows(cx<T>* buf, const cx<T>* tw, const FftPlan& pl, int es, int nrows,
                                         int n0, int s0, int s1) {
    int p = 1;
    for (int s = 0; s < pl.nst; ++s) {
        const int r = pl.rad[s];
        if (r == 2)
            fft_stage<2, EPT, T, INV>(buf, tw, pl.n, p, es, nrows, n0, s0, s1);
        else if (r == 3)
            fft_stage<3, EPT, T, INV>(buf, tw, pl.n, p, es, nrows, n0, s0, s1);
        else if (r == 4)
            fft_stage<4, EPT, T, INV>(buf, tw, pl.n, p, es, nrows, n0, s0, s1);
        else
            fft_stage<8, EPT, T, INV>(buf, tw, pl.n, p, es, nrows, n0, s0, s1);
        p *= r;
    }
}

}  // namespace gf

// ------------------------------------------------ compile-time specialisation
// The same Stockham stages with the transform length, radix sequence, row
// geometry and thread count known at compile time, so that every index
// division and modulo becomes a shift or multiply and every loop unrolls.
namespace gf {

constexpr int ct_nst(int n) {
    int s = 0, m = n;
    while (m % 3 == 0) {
        ++s;
        m /= 3;
    }
    int a = 0;
    while (m % 2 == 0) {
        ++a;
        m /= 2;
    }
    while (a >= 3 && a != 4) {
        ++s;
        a -= 3;
    }
    while (a >= 2) {
        ++s;
        a -= 2;
    }
    if (a == 1) ++s;
    return s;
}

constexpr int ct_rad(int n, int idx) {
    int r[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int s = 0, m = n;
    while (m % 3 == 0) {
        r[s++] = 3;
        m /= 3;
    }
    int a = 0;
    while (m % 2 == 0) {
        ++a;
        m /= 2;
    }
    while (a >= 3 && a != 4) {
        r[s++] = 8;
        a -= 3;
    }
    while (a >= 2) {
        r[s++] = 4;
        a -= 2;
    }
    if (a == 1) r[s++] = 2;
    return r[idx];
}

// Geometry of a batch of rows: row b starts at (b % N0)*S0 + (b / N0)*S1,
// elements ES apart.
template <int NROWS, int ES, int N0, int S0, int S1>
struct Rows {
    static constexpr int nrows = NROWS, es = ES, n0 = N0, s0 = S0, s1 = S1;
};

// Where a stage reads its inputs and puts its outputs: element e of row b. The LDS forms address
// row b at (b % n0)*s0 + (b / n0)*s1 with elements es apart.
template <class RW, typename T>
struct LdsIo {
    cx<T>* buf;
    static constexpr bool lds_in = true, lds_out = true;
    __device__ __forceinline__ int at(int b, int e) const {
        return (b % RW::n0) * RW::s0 + (b / RW::n0) * RW::s1 + e * RW::es;
    }
    __device__ __forceinline__ cx<T> ld(int b, int e) const { return buf[at(b, e)]; }
    __device__ __forceinline__ void st(int b, int e, cx<T> v) const { buf[at(b, e)] = v; }
};

// One radix-R stage in three steps, on the butterflies thread tid takes (PER of them): load the
// inputs of each from IN, multiply them by the twiddles, then take the R-point DFTs and put the
// outputs to OUT.
template <int N, int R, class RW, int NT>
struct StageShape {
    static constexpr int M = N / R, ITEMS = RW::nrows * M, PER = (ITEMS + NT - 1) / NT;
    __device__ __forceinline__ static bool valid(int tid, int it) { return ITEMS % NT == 0 || tid + it * NT < ITEMS; }
    __device__ __forceinline__ static int row(int tid, int it) { return (tid + it * NT) % RW::nrows; }
    __device__ __forceinline__ static int item(int tid, int it) { return (tid + it * NT) / RW::nrows; }
};

// A thread's butterfly inputs for one stage.
template <int N, int R, class RW, int NT, typename T>
using StageRegs = cx<T>[StageShape<N, R, RW, NT>::PER][R];

template <int N, int R, class RW, int NT, typename T, class IN>
__device__ __forceinline__ void stage_load(const IN& in, StageRegs<N, R, RW, NT, T>& v, int tid) {
    using SS = StageShape<N, R, RW, NT>;
#pragma unroll
    for (int it = 0; it < SS::PER; ++it) {
        if (SS::valid(tid, it)) {
            const int b = SS::row(tid, it), i = SS::item(tid, it);
#pragma unroll
            for (int j = 0; j < R; ++j) v[it][j] = in.ld(b, i + j * SS::M);
        }
    }
}

template <int N, int R, int P, class RW, int NT, typename T, bool INV>
__device__ __forceinline__ void stage_twiddle(const cx<T>* tw, StageRegs<N, R, RW, NT, T>& v, int tid) {
    using SS = StageShape<N, R, RW, NT>;
    if constexpr (P > 1) {  // the first stage's twiddles are all 1
        constexpr int TWSTEP = N / (P * R);
#pragma unroll
        for (int it = 0; it < SS::PER; ++it) {
            if (SS::valid(tid, it)) {
                const int k = SS::item(tid, it) % P;
#pragma unroll
                for (int j = 1; j < R; ++j) {
                    cx<T> t = tw[j * k * TWSTEP];
                    if (INV) t.im = -t.im;
                    v[it][j] = cmul(v[it][j], t);
                }
            }
        }
    }
}

template <int N, int R, int P, class RW, int NT, typename T, bool INV, class OUT>
__device__ __forceinline__ void stage_store(StageRegs<N, R, RW, NT, T>& v, const OUT& out, int tid) {
    using SS = StageShape<N, R, RW, NT>;
#pragma unroll
    for (int it = 0; it < SS::PER; ++it) {
        if (SS::valid(tid, it)) {
            const int b = SS::row(tid, it), i = SS::item(tid, it);
            const int k = i % P;
            dft_small<R, T, INV>(v[it]);
#pragma unroll
            for (int j = 0; j < R; ++j) out.st(b, (i - k) * R + k + j * P, v[it][j]);
        }
    }
}

// The whole stage. A block barrier separates the reads from the writes only when both are in
// LDS, and follows the writes only when they go to LDS.
template <int N, int R, int P, class RW, int NT, typename T, bool INV, class IN, class OUT>
__device__ __forceinline__ void fft_stage_io(const cx<T>* tw, const IN& in, const OUT& out, int tid) {
    StageRegs<N, R, RW, NT, T> v;
    stage_load<N, R, RW, NT, T>(in, v, tid);
    stage_twiddle<N, R, P, RW, NT, T, INV>(tw, v, tid);
    if constexpr (IN::lds_in && OUT::lds_out) __syncthreads();
    stage_store<N, R, P, RW, NT, T, INV>(v, out, tid);
    if constexpr (OUT::lds_out) __syncthreads();
}

// Radix of stage S of a length-N transform whose radices are taken in the order ct_rad gives
// (REV false) or in the reverse order (REV true). Either order is a valid Stockham sequence.
template <int N, bool REV>
constexpr int stage_radix(int S) {
    return ct_rad(N, REV ? ct_nst(N) - 1 - S : S);
}

// Stages S .. SEND-1 of a batch of rows (P the product of the radices before S): stage S0 (the
// first of the range) reads from FIRST, stage SEND-1 writes to LAST, the others work in LDS.
template <int N, int S0, int S, int SEND, int P, bool REV, class RW, int NT, typename T, bool INV, class FIRST,
          class LAST>
__device__ __forceinline__ void fft_stages_io(cx<T>* buf, const cx<T>* tw, const FIRST& first, const LAST& last,
                                              int tid) {
    if constexpr (S < SEND) {
        constexpr int R = stage_radix<N, REV>(S);
        const LdsIo<RW, T> lds{buf};
        if constexpr (S == S0 && S + 1 == SEND)
            fft_stage_io<N, R, P, RW, NT, T, INV>(tw, first, last, tid);
        else if constexpr (S == S0)
            fft_stage_io<N, R, P, RW, NT, T, INV>(tw, first, lds, tid);
        else if constexpr (S + 1 == SEND)
            fft_stage_io<N, R, P, RW, NT, T, INV>(tw, lds, last, tid);
        else
            fft_stage_io<N, R, P, RW, NT, T, INV>(tw, lds, lds, tid);
        fft_stages_io<N, S0, S + 1, SEND, P * R, REV, RW, NT, T, INV>(buf, tw, first, last, tid);
    }
}

// All stages of a batch of rows: the first stage reads from FIRST, the last writes to LAST, the
// others work in LDS.
template <int N, int S, int P, class RW, int NT, typename T, bool INV, class FIRST, class LAST>
__device__ __forceinline__ void fft_rows_io(cx<T>* buf, const cx<T>* tw, const FIRST& first, const LAST& last,
                                            int tid) {
    fft_stages_io<N, S, S, ct_nst(N), P, false, RW, NT, T, INV>(buf, tw, first, last, tid);
}

template <int N, int S, int P, class RW, int NT, typename T, bool INV>
__device__ __forceinline__ void fft_rows_ct(cx<T>* buf, const cx<T>* tw) {
    const LdsIo<RW, T> lds{buf};
    fft_rows_io<N, S, P, RW, NT, T, INV>(buf, tw, lds, lds, threadIdx.x);
}

// Forward transform of a batch of rows in LDS, a per-element map F on the spectrum, and the
// inverse transform back into LDS. The inverse takes the radices in the reverse order: its first
// stage then reads exactly the elements the forward's last stage leaves in a thread's registers
// (stage with p*R = N writes element i + j*p of its butterfly i, and the reversed first stage,
// m = N/R = p, reads element i + j*m), so F and that stage run on those registers and the two
// stages share one LDS exchange. F is called as F.apply(row, element, value).
template <int N, class RW, int NT, typename T, class F>
__device__ __forceinline__ void fft_rows_map_inverse(cx<T>* buf, const cx<T>* tw, const F& fmap, int tid) {
    constexpr int NS = ct_nst(N), RL = ct_rad(N, NS - 1), PL = N / RL;
    using SS = StageShape<N, RL, RW, NT>;
    const LdsIo<RW, T> lds{buf};
    fft_stages_io<N, 0, 0, NS - 1, 1, false, RW, NT, T, false>(buf, tw, lds, lds, tid);
    StageRegs<N, RL, RW, NT, T> v;
    stage_load<N, RL, RW, NT, T>(lds, v, tid);
    stage_twiddle<N, RL, PL, RW, NT, T, false>(tw, v, tid);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < SS::PER; ++it) {
        if (SS::valid(tid, it)) {
            const int b = SS::row(tid, it), i = SS::item(tid, it);
            dft_small<RL, T, false>(v[it]);
#pragma unroll
            for (int j = 0; j < RL; ++j) v[it][j] = fmap.apply(b, i + j * PL, v[it][j]);
            dft_small<RL, T, true>(v[it]);
#pragma unroll
            for (int j = 0; j < RL; ++j) lds.st(b, i * RL + j, v[it][j]);
        }
    }
    __syncthreads();
    fft_stages_io<N, 1, 1, NS, RL, true, RW, NT, T, true>(buf, tw, lds, lds, tid);
}

}  // namespace gf

// Learned spectral preconditioner: recording, inference table and training.
//
// The fixed Fourier-acceleration multiplier m0(p) = (alpha/2) p2max / p^2(p)
// (divided by V for the unnormalised transforms) is replaced by
//     m(p) = m0(p) * exp(o_s(p) + o_a(0)),
// where (o_s, o_a) are the outputs of a 6 -> 64 -> 64 -> 2 tanh network on the
// features of each distinct momentum tuple n_mu in [0, N_mu/2] (p^2 is even
// in every n_mu): x = (p^2_mu/4 - 1/2 for mu = 0..3, log10(theta_k)/8 + 1,
// k/64). o_a at the zero tuple sets a global step; all-zero outputs give the
// fixed multiplier exactly. Parameters (float): W1 (64x6), b1, W2 (64x64), b2,
// W3 (2x64), b3.
//
// Training signal, recorded on plain-FA trajectories: per tuple,
// P_k = sum over the +-n reflections and the four packed fields of |Z(p)|^2
// after the forward FFT, and C_k = the same sum of Re[Z_{k+1}(p) conj(Z_k(p))].
// Loss of one sample: sum_p P (1 - m kappa)^2 / sum_p P with
// kappa = (1 - C/P)/m0, the observed response of each mode.
#pragma once

#include "gf_device.hpp"

namespace gf {

constexpr int kMlpIn = 6, kMlpH = 64, kMlpOut = 2;
constexpr int kMlpParams = kMlpH * kMlpIn + kMlpH + kMlpH * kMlpH + kMlpH + kMlpOut * kMlpH + kMlpOut;
constexpr double kRatioFloor = 1e-12;  // the training loss is ln(max(predicted residual ratio, this))
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kMlpH * kMlpIn, kOffW2 = kOffB1 + kMlpH, kOffB2 = kOffW2 + kMlpH * kMlpH,
              kOffW3 = kOffB2 + kMlpH, kOffB3 = kOffW3 + kMlpOut * kMlpH;

// Folded tuple index (first axis fastest) of the mode n of a lattice.
__device__ __forceinline__ int fold1(int n, int N) { return n <= N / 2 ? n : N - n; }

struct TupleGeom {
    int n[4];   // lattice extents
    int h[4];   // N_mu/2 + 1
    int count;  // number of tuples
};

__device__ __forceinline__ int tuple_index(const TupleGeom& tg, int nx, int ny, int nz, int nt) {
    return fold1(nx, tg.n[0]) + tg.h[0] * (fold1(ny, tg.n[1]) + tg.h[1] * (fold1(nz, tg.n[2]) + tg.h[2] * fold1(nt, tg.n[3])));
}

// -------------------------------------------------------------- recording
// Per tuple, summed over the tuple's +-n reflections and the four packed
// fields (full 4D spectra, planes ps apart): out[3i] = P = |Sk|^2,
// out[3i+1] = C = Re Sk1 conj(Sk) (Sk1: after the plain step),
// out[3i+2] = E = |Sp|^2 (Sp: after the probe step). Double.
template <typename T>
__global__ void __launch_bounds__(256) k_record_tuples(const cx<T>* __restrict__ Sk, const cx<T>* __restrict__ Sk1,
                                                       const cx<T>* __restrict__ Sp, size_t ps, TupleGeom tg,
                                                       double* __restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= tg.count) return;
    int t[4], r = i;
    for (int m = 0; m < 4; ++m) {
        t[m] = r % tg.h[m];
        r /= tg.h[m];
    }
    double P = 0.0, C = 0.0, E = 0.0;
    for (int a = 0; a < 16; ++a) {
        int q[4];
        bool dup = false;
        for (int m = 0; m < 4; ++m) {
            const int flip = (a >> m) & 1;
            q[m] = flip ? (tg.n[m] - t[m]) % tg.n[m] : t[m];
            if (flip && q[m] == t[m]) dup = true;  // the reflection is the mode itself
        }
        if (dup) continue;
        const size_t s = (size_t)q[0] + (size_t)tg.n[0] * (q[1] + (size_t)tg.n[1] * (q[2] + (size_t)tg.n[2] * q[3]));
        for (int f = 0; f < 4; ++f) {
            const cx<T> z0 = Sk[(size_t)f * ps + s], z1 = Sk1[(size_t)f * ps + s], zp = Sp[(size_t)f * ps + s];
            P += (double)z0.re * z0.re + (double)z0.im * z0.im;
            C += (double)z1.re * z0.re + (double)z1.im * z0.im;
            E += (double)zp.re * zp.re + (double)zp.im * zp.im;
        }
    }
    out[3 * i] = P;
    out[3 * i + 1] = C;
    out[3 * i + 2] = E;
}

// ------------------------------------------------------------ inference
__device__ __forceinline__ void mlp_features(const float* sin2_4, float log10_theta, float k, float x[kMlpIn]) {
#pragma unroll
    for (int m = 0; m < 4; ++m) x[m] = sin2_4[m] * 0.25f - 0.5f;
    x[4] = log10_theta * 0.125f + 1.0f;
    x[5] = k * (1.0f / 64.0f);
}

// Multiplier table for the current iteration: mtab[i] = coef / p^2 *
// exp(o_s(i) + o_a(0)) (coef = (alpha/2) p2max / V), 0 at the zero tuple;
// theta and the iteration count come from the control block. The hidden
// layer 64 x 64 is a dense contraction over the tuples and runs on the matrix
// cores: a wave takes kTableGroups groups of 16 tuples; for each, every lane
// evaluates layer 1 for the 16 hidden units k = l/16 + 4m of tuple l%16 (its
// A operand), v_mfma_f32_16x16x4f32 forms the 16 x 64 pre-activations of
// layer 2 in four 16 x 16 tiles over K = 64 (16 steps, B operands read from
// the padded W2 in LDS), and layer 3 is a sum across the 16 lanes that hold
// one tuple's hidden units. o_a is evaluated once per block at the zero
// tuple, one hidden unit per lane of wave 0. (Keeping the B operands in
// registers for several groups measured slower: 256 VGPRs, one wave per SIMD.)
typedef float f32x4 __attribute__((ext_vector_type(4)));

// tanh(x) = 1 - 2 / (exp(2x) + 1) with the hardware exponential and
// reciprocal: absolute error about 1e-7, saturating correctly at both ends
// (inference only; the training kernels use tanhf).
__device__ __forceinline__ float tanh_fast(float x) {
    return 1.0f - 2.0f * __frcp_rn(__expf(2.0f * x) + 1.0f);
}
constexpr int kTableGroups = 1;
constexpr int kTableTuplesPerBlock = 4 * 16 * kTableGroups;

template <typename T>
__global__ void __launch_bounds__(256) k_mlp_table(const float* __restrict__ params, const T* __restrict__ sin2,
                                                   TupleGeom tg, double coef, const Ctl* __restrict__ ctl,
                                                   int force, T* __restrict__ mtab) {
    if (!force && ctl->done) return;
    constexpr int W2S = kMlpH + 1;  // padded row stride of W2 in LDS
    __shared__ float w1[kMlpH * kMlpIn], b1[kMlpH], w2[kMlpH * W2S], b2[kMlpH], w3[2 * kMlpH], h1z[kMlpH];
    __shared__ float c1[kMlpH];  // b1 + the theta and k terms of layer 1, shared by every tuple
    __shared__ float oa_s;
    {
        // every load first, then the LDS stores: one memory round trip for the whole network
        constexpr int N2 = kMlpH * kMlpH / 256, N1 = (kMlpH * kMlpIn + 255) / 256;
        float r2[N2], r1[N1], rb1 = 0.f, rb2 = 0.f, rw30 = 0.f, rw31 = 0.f;
#pragma unroll
        for (int q = 0; q < N2; ++q) r2[q] = params[kOffW2 + q * 256 + threadIdx.x];
#pragma unroll
        for (int q = 0; q < N1; ++q) {
            const int i = q * 256 + threadIdx.x;
            r1[q] = i < kMlpH * kMlpIn ? params[kOffW1 + i] : 0.f;
        }
        if (threadIdx.x < kMlpH) {
            rb1 = params[kOffB1 + threadIdx.x];
            rb2 = params[kOffB2 + threadIdx.x];
            rw30 = params[kOffW3 + threadIdx.x];
            rw31 = params[kOffW3 + kMlpH + threadIdx.x];
        }
#pragma unroll
        for (int q = 0; q < N2; ++q) {
            const int i = q * 256 + threadIdx.x;
            w2[(i / kMlpH) * W2S + i % kMlpH] = r2[q];
        }
#pragma unroll
        for (int q = 0; q < N1; ++q) {
            const int i = q * 256 + threadIdx.x;
            if (i < kMlpH * kMlpIn) w1[i] = r1[q];
        }
        if (threadIdx.x < kMlpH) {
            b1[threadIdx.x] = rb1;
            b2[threadIdx.x] = rb2;
            w3[threadIdx.x] = rw30;
            w3[kMlpH + threadIdx.x] = rw31;
        }
    }
    __syncthreads();
    const float lt = (float)log10(fmax(ctl->theta, 1e-300));
    const float kk = (float)ctl->iters;
    const float b30 = params[kOffB3], b31 = params[kOffB3 + 1];
    if (threadIdx.x < kMlpH) {  // o_a: layer 1 of the zero tuple
        const int j = threadIdx.x;
        float zx[kMlpIn];
        const float zs[4] = {0.f, 0.f, 0.f, 0.f};
        mlp_features(zs, lt, kk, zx);
        const float cj = fmaf(w1[j * kMlpIn + 5], zx[5], fmaf(w1[j * kMlpIn + 4], zx[4], b1[j]));
        c1[j] = cj;
        float a = cj;
#pragma unroll
        for (int i = 0; i < 4; ++i) a = fmaf(w1[j * kMlpIn + i], zx[i], a);
        h1z[j] = tanh_fast(a);
    }
    __syncthreads();
    if (threadIdx.x < kMlpH) {  // layers 2 and 3 of the zero tuple, second output
        const int j = threadIdx.x;
        float a0 = b2[j], a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
        for (int i = 0; i < kMlpH; i += 4) {
            a0 = fmaf(w2[j * W2S + i], h1z[i], a0);
            a1 = fmaf(w2[j * W2S + i + 1], h1z[i + 1], a1);
            a2 = fmaf(w2[j * W2S + i + 2], h1z[i + 2], a2);
            a3 = fmaf(w2[j * W2S + i + 3], h1z[i + 3], a3);
        }
        float p = w3[kMlpH + j] * tanh_fast((a0 + a1) + (a2 + a3));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) p += __shfl_xor(p, o, 64);
        if (j == 0) oa_s = p + b31;
    }
    __syncthreads();
    const double oa = (double)oa_s;
    const int l = threadIdx.x & 63, kq = l >> 4, lc = l & 15;
    // B operands: W2[unit n*16 + lc][input 4m + kq]
    const T* sx = sin2;
    const T* sy = sx + tg.n[0];
    const T* sz = sy + tg.n[1];
    const T* st = sz + tg.n[2];
    for (int grp = 0; grp < kTableGroups; ++grp) {
        const int t0 = blockIdx.x * kTableTuplesPerBlock + ((threadIdx.x >> 6) * kTableGroups + grp) * 16;
        // layer 1 for tuple t0 + lc, hidden units kq + 4m
        int ti = t0 + lc;
        if (ti >= tg.count) ti = 0;
        int c4[4], r = ti;
        for (int m = 0; m < 4; ++m) {
            c4[m] = r % tg.h[m];
            r /= tg.h[m];
        }
        const float s4[4] = {(float)sx[c4[0]], (float)sy[c4[1]], (float)sz[c4[2]], (float)st[c4[3]]};
        float x[kMlpIn];
        mlp_features(s4, lt, kk, x);
        float h1[16];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int j = kq + 4 * m;
            float a = c1[j];
#pragma unroll
            for (int i = 0; i < 4; ++i) a = fmaf(w1[j * kMlpIn + i], x[i], a);
            h1[m] = tanh_fast(a);
        }
        // layer 2: acc[n] holds rows 4*kq + q (tuples t0 + 4*kq + q), unit n*16 + lc
        f32x4 acc[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            acc[n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int m = 0; m < 16; ++m) acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(h1[m], w2[(n * 16 + lc) * W2S + 4 * m + kq], acc[n], 0, 0, 0);
        }
        // layer 3, first output: partial sums over this lane's units, then over the 16 lanes of the group
        float o0[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const int j = n * 16 + lc;
#pragma unroll
            for (int q = 0; q < 4; ++q) o0[q] = fmaf(w3[j], tanh_fast(acc[n][q] + b2[j]), o0[q]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int o = 1; o < 16; o <<= 1) o0[q] += __shfl_xor(o0[q], o, 64);
        if (lc < 4) {
            const int t = t0 + 4 * kq + lc;
            const float os = lc == 0 ? o0[0] : lc == 1 ? o0[1] : lc == 2 ? o0[2] : o0[3];
            if (t < tg.count) {
                int r2 = t, d4[4];
                for (int m = 0; m < 4; ++m) {
                    d4[m] = r2 % tg.h[m];
                    r2 /= tg.h[m];
                }
                const double p2 = (double)sx[d4[0]] + (double)sy[d4[1]] + (double)sz[d4[2]] + (double)st[d4[3]];
                mtab[t] = p2 > 0.0 ? (T)(coef / p2 * exp((double)(os + b30) + oa)) : T(0);
            }
        }
    }
}

// --------------------------------------------------------------- training
// Samples from records: record r holds (P_r, C_r, E_r) per tuple, E_r the
// energy after the probe step (every multiplier times sigma). Sample s uses
// record r = first + s*every and the next one: row s*T + i gets the features
// of tuple i at (theta[r], iteration k0 + r) and the coefficients (a, b, c)
// of the quadratic e(x) = a - 2 b x + c x^2 through the residual energies
// e(0) = P_r, e(sigma) = E_r and e(1) = P_{r+1}, with c raised to b^2/a where
// needed so that e stays >= 0; formed in double.
__global__ void __launch_bounds__(256) k_make_samples(const double* __restrict__ rec, const double* __restrict__ theta,
                                                      int first, int every, long long k0, double sigma,
                                                      int64_t nrows, TupleGeom tg, float* __restrict__ X,
                                                      float* __restrict__ tgt) {
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= nrows) return;
    const int s = (int)(row / tg.count), i = (int)(row % tg.count);
    const int64_t r = (int64_t)first + (int64_t)s * every;
    int t[4], q = i;
    for (int m = 0; m < 4; ++m) {
        t[m] = q % tg.h[m];
        q /= tg.h[m];
    }
    float s4[4];
    for (int m = 0; m < 4; ++m) {
        const double sv = sinpi((double)t[m] / (double)tg.n[m]);
        s4[m] = (float)(4.0 * sv * sv);
    }
    float x[kMlpIn];
    mlp_features(s4, (float)log10(fmax(theta[r], 1e-300)), (float)(k0 + r), x);
#pragma unroll
    for (int c = 0; c < kMlpIn; ++c) X[row * kMlpIn + c] = x[c];
    const double P = rec[(r * tg.count + i) * 3], E = rec[(r * tg.count + i) * 3 + 2];
    const double Pn = rec[((r + 1) * tg.count + i) * 3];
    const double v = (E - P - sigma * (Pn - P)) / (sigma * sigma - sigma);
    const double b = -0.5 * (Pn - P - v);
    const double c = P > 0.0 ? fmax(v, b * b / P) : v;
    tgt[row * 3] = (float)P;
    tgt[row * 3 + 1] = (float)b;
    tgt[row * 3 + 2] = (float)c;
}

// Rows are momentum tuples of samples; sample s owns rows [off[s], off[s+1]),
// its first row being the zero tuple. tgt row = (m0, P, kappa).

// Forward pass keeping the activations: H1, H2 (n x 64), O (n x 2).
__global__ void __launch_bounds__(256) k_mlp_forward(const float* __restrict__ params, const float* __restrict__ X,
                                                     int64_t n, float* __restrict__ H1, float* __restrict__ H2,
                                                     float* __restrict__ O) {
    __shared__ float w[kMlpParams];
    for (int i = threadIdx.x; i < kMlpParams; i += 256) w[i] = params[i];
    __syncthreads();
    const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (row >= n) return;
    float x[kMlpIn];
#pragma unroll
    for (int i = 0; i < kMlpIn; ++i) x[i] = X[row * kMlpIn + i];
    float h1[kMlpH];
#pragma unroll
    for (int j = 0; j < kMlpH; ++j) {
        float a = w[kOffB1 + j];
#pragma unroll
        for (int i = 0; i < kMlpIn; ++i) a = fmaf(w[kOffW1 + j * kMlpIn + i], x[i], a);
        h1[j] = tanhf(a);
        H1[(int64_t)j * n + row] = h1[j];  // column-major: the lanes' consecutive rows store contiguously
    }
    float a0 = w[kOffB3], a1 = w[kOffB3 + 1];
    for (int j = 0; j < kMlpH; ++j) {
        float a = w[kOffB2 + j];
#pragma unroll
        for (int i = 0; i < kMlpH; ++i) a = fmaf(w[kOffW2 + j * kMlpH + i], h1[i], a);
        const float h2 = tanhf(a);
        H2[(int64_t)j * n + row] = h2;
        a0 = fmaf(w[kOffW3 + j], h2, a0);
        a1 = fmaf(w[kOffW3 + kMlpH + j], h2, a1);
    }
    O[row * 2] = a0;
    O[row * 2 + 1] = a1;
}

// One block per sample: loss (double) and dL/dO for the sample's rows, the
// mean over ns samples. dO is written for every row (o_a only at row 0).
__global__ void __launch_bounds__(256) k_mlp_loss(const float* __restrict__ O, const float* __restrict__ tgt,
                                                  const int* __restrict__ off, int ns, float* __restrict__ dO,
                                                  double* __restrict__ sample_loss) {
    const int smp = blockIdx.x;
    const int r0 = off[smp], r1 = off[smp + 1];
    const double oa = O[(int64_t)r0 * 2 + 1];
    __shared__ double red[4][256 / 64];
    double asum = 0.0, lsum = 0.0;
    for (int r = r0 + threadIdx.x; r < r1; r += 256) {
        const double a = tgt[(int64_t)r * 3], b = tgt[(int64_t)r * 3 + 1], c = tgt[(int64_t)r * 3 + 2];
        const double s = exp((double)O[(int64_t)r * 2] + oa);
        asum += a;
        lsum += a - 2.0 * s * b + s * s * c;
    }
    asum = wave_sum(asum);
    lsum = wave_sum(lsum);
    const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) {
        red[0][wv] = asum;
        red[1][wv] = lsum;
    }
    __syncthreads();
    double Atot = 0.0, Ltot = 0.0;
    for (int i = 0; i < 256 / 64; ++i) {
        Atot += red[0][i];
        Ltot += red[1][i];
    }
    // loss = ln(Ltot / Atot), floored at ln(kRatioFloor) with zero gradient there;
    // d loss/ds = (2 s c - 2 b) / (Ltot ns); do_s = d loss/ds * s; do_a(row 0) = sum over rows
    const bool floored = !(Ltot / Atot > kRatioFloor);
    double gsum = 0.0;
    for (int r = r0 + threadIdx.x; r < r1; r += 256) {
        const double b = tgt[(int64_t)r * 3 + 1], c = tgt[(int64_t)r * 3 + 2];
        const double s = exp((double)O[(int64_t)r * 2] + oa);
        const double g = floored ? 0.0 : (2.0 * s * c - 2.0 * b) / (Ltot * ns) * s;
        dO[(int64_t)r * 2] = (float)g;
        dO[(int64_t)r * 2 + 1] = 0.0f;
        gsum += g;
    }
    gsum = wave_sum(gsum);
    __syncthreads();
    if (l == 0) red[2][wv] = gsum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < 256 / 64; ++i) t += red[2][i];
        dO[(int64_t)r0 * 2 + 1] = (float)t;
        sample_loss[smp] = log(floored ? kRatioFloor : Ltot / Atot);
    }
}

// Backward pass. Block b walks kBwdChunks chunks of kBwdRows consecutive rows (kBwdBlockRows in all).
// Per chunk the rows' hidden activations, inputs and output gradients are staged in LDS; eight threads
// per row form 8 entries each of dz2 = (dO W3) (1 - h2^2) and then of dz1 = (dz2 W2) (1 - h1^2). Every thread
// then adds, rows in order, its 4 x 4 tile of dW2 = sum_r dz2[r] h1[r]^T and up to three of the other
// 642 parameters to register accumulators. The block's partial gradient (float) goes to gpart[b];
// k_grad_reduce adds the partials in block order, in double. Activations are column-major (H[j * n + row]).
constexpr int kBwdRows = 32;
constexpr int kBwdChunks = 16;
constexpr int kBwdTpr = 256 / kBwdRows;  // threads per row in the delta phase
constexpr int kBwdPer = kMlpH / kBwdTpr;  // dz1 entries per thread
constexpr int kBwdBlockRows = kBwdRows * kBwdChunks;
constexpr int kBwdStride = kMlpH + 4;  // LDS row stride: 16-byte aligned rows for the tile loads
constexpr int kBwdOther = kMlpParams - kMlpH * kMlpH;  // W1, b1, b2, W3, b3
constexpr size_t kBwdLds =
    (size_t)(kMlpH * kMlpH + kMlpOut * kMlpH + 4 * kBwdRows * kBwdStride + kBwdRows * kMlpIn + kBwdRows * kMlpOut) *
    sizeof(float);

__device__ __forceinline__ float bwd_other_term(int p, int r, const float* dz1s, const float* dz2s, const float* xs,
                                                const float* dOs, const float* h2s) {
    // p indexes the parameters outside W2 in the order W1, b1, b2, W3, b3
    if (p < kMlpH * kMlpIn) return dz1s[r * kBwdStride + p / kMlpIn] * xs[r * kMlpIn + p % kMlpIn];
    p -= kMlpH * kMlpIn;
    if (p < kMlpH) return dz1s[r * kBwdStride + p];
    p -= kMlpH;
    if (p < kMlpH) return dz2s[r * kBwdStride + p];
    p -= kMlpH;
    if (p < kMlpOut * kMlpH) return dOs[r * kMlpOut + p / kMlpH] * h2s[r * kBwdStride + p % kMlpH];
    p -= kMlpOut * kMlpH;
    return dOs[r * kMlpOut + p];
}

__device__ __forceinline__ int bwd_other_offset(int p) {
    if (p < kMlpH * kMlpIn) return kOffW1 + p;
    p -= kMlpH * kMlpIn;
    if (p < kMlpH) return kOffB1 + p;
    p -= kMlpH;
    if (p < kMlpH) return kOffB2 + p;
    p -= kMlpH;
    if (p < kMlpOut * kMlpH) return kOffW3 + p;
    return kOffB3 + (p - kMlpOut * kMlpH);
}

__global__ void __launch_bounds__(256) k_mlp_backward(const float* __restrict__ params, const float* __restrict__ X,
                                                      const float* __restrict__ H1, const float* __restrict__ H2,
                                                      const float* __restrict__ dO, int64_t n,
                                                      float* __restrict__ gpart) {
    extern __shared__ __align__(16) float lds[];
    float* w2 = lds;                                  // [j][i]
    float* w3 = w2 + kMlpH * kMlpH;                   // [o][j]
    float* h1s = w3 + kMlpOut * kMlpH;                // [r][i], stride kBwdStride
    float* dz2s = h1s + kBwdRows * kBwdStride;        // [r][j]
    float* dz1s = dz2s + kBwdRows * kBwdStride;       // [r][i]
    float* h2s = dz1s + kBwdRows * kBwdStride;        // [r][j]
    float* xs = h2s + kBwdRows * kBwdStride;          // [r][k]
    float* dOs = xs + kBwdRows * kMlpIn;              // [r][o]
    const int t = threadIdx.x;
    for (int i = t; i < kMlpH * kMlpH; i += 256) w2[i] = params[kOffW2 + i];
    for (int i = t; i < kMlpOut * kMlpH; i += 256) w3[i] = params[kOffW3 + i];
    const int j0 = (t >> 4) * 4, i0 = (t & 15) * 4;  // this thread's tile of dW2
    float acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.f;
    float oacc[3] = {0.f, 0.f, 0.f};
    const int64_t blk0 = (int64_t)blockIdx.x * kBwdBlockRows;
    for (int ch = 0; ch < kBwdChunks; ++ch) {
        const int64_t row0 = blk0 + (int64_t)ch * kBwdRows;
        if (row0 >= n) break;  // uniform over the block
        __syncthreads();  // the previous chunk's LDS reads are done
        {  // H1, H2 column-major -> h1s[r][i], h2s[r][j]: every load issued before the LDS stores
            constexpr int PER = kMlpH * kBwdRows / 256;
            float v1[PER], v2[PER];
#pragma unroll
            for (int m = 0; m < PER; ++m) {
                const int e = t + 256 * m;
                const int i = e / kBwdRows, r = e % kBwdRows;
                const int64_t row = row0 + r;
                v1[m] = row < n ? H1[(int64_t)i * n + row] : 0.f;
                v2[m] = row < n ? H2[(int64_t)i * n + row] : 0.f;
            }
#pragma unroll
            for (int m = 0; m < PER; ++m) {
                const int e = t + 256 * m;
                const int i = e / kBwdRows, r = e % kBwdRows;
                h1s[r * kBwdStride + i] = v1[m];
                h2s[r * kBwdStride + i] = v2[m];
            }
        }
        for (int e = t; e < kBwdRows * kMlpIn; e += 256) {
            const int64_t idx = row0 * kMlpIn + e;
            xs[e] = idx < n * kMlpIn ? X[idx] : 0.f;
        }
        for (int e = t; e < kBwdRows * kMlpOut; e += 256) {
            const int64_t idx = row0 * kMlpOut + e;
            dOs[e] = idx < n * kMlpOut ? dO[idx] : 0.f;
        }
        __syncthreads();
        {  // kBwdTpr threads per row, kBwdPer entries each: first dz2, then (after the barrier) dz1
            const int r = t / kBwdTpr, q = t % kBwdTpr;
            const float d0 = dOs[r * kMlpOut], d1 = dOs[r * kMlpOut + 1];
#pragma unroll
            for (int jj = 0; jj < kBwdPer; ++jj) {
                const int j = q * kBwdPer + jj;
                const float h2 = h2s[r * kBwdStride + j];
                dz2s[r * kBwdStride + j] = (d0 * w3[j] + d1 * w3[kMlpH + j]) * (1.f - h2 * h2);
            }
            __syncthreads();
            float a[kBwdPer];
#pragma unroll
            for (int ii = 0; ii < kBwdPer; ++ii) a[ii] = 0.f;
#pragma unroll 8
            for (int j = 0; j < kMlpH; ++j) {
                const float dz = dz2s[r * kBwdStride + j];
                const float4* wr = reinterpret_cast<const float4*>(w2 + j * kMlpH + q * kBwdPer);
#pragma unroll
                for (int v = 0; v < kBwdPer / 4; ++v) {
                    const float4 wv = wr[v];
                    a[4 * v] = fmaf(dz, wv.x, a[4 * v]);
                    a[4 * v + 1] = fmaf(dz, wv.y, a[4 * v + 1]);
                    a[4 * v + 2] = fmaf(dz, wv.z, a[4 * v + 2]);
                    a[4 * v + 3] = fmaf(dz, wv.w, a[4 * v + 3]);
                }
            }
#pragma unroll
            for (int ii = 0; ii < kBwdPer; ++ii) {
                const int i = q * kBwdPer + ii;
                const float h1 = h1s[r * kBwdStride + i];
                dz1s[r * kBwdStride + i] = a[ii] * (1.f - h1 * h1);
            }
        }
        __syncthreads();
#pragma unroll 4
        for (int r = 0; r < kBwdRows; ++r) {  // rows in order (a full unroll would hoist every row's loads)
            const float4 dz = *reinterpret_cast<const float4*>(dz2s + r * kBwdStride + j0);
            const float4 hv = *reinterpret_cast<const float4*>(h1s + r * kBwdStride + i0);
            const float dzv[4] = {dz.x, dz.y, dz.z, dz.w}, hh[4] = {hv.x, hv.y, hv.z, hv.w};
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = fmaf(dzv[a], hh[b], acc[a][b]);
        }
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int p = t + 256 * m;
            if (p < kBwdOther)
#pragma unroll 4
                for (int r = 0; r < kBwdRows; ++r)
                    oacc[m] += bwd_other_term(p, r, dz1s, dz2s, xs, dOs, h2s);
        }
    }
    float* gp = gpart + (size_t)blockIdx.x * kMlpParams;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) gp[kOffW2 + (j0 + a) * kMlpH + i0 + b] = acc[a][b];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const int p = t + 256 * m;
        if (p < kBwdOther) gp[bwd_other_offset(p)] = oacc[m];
    }
}

__global__ void __launch_bounds__(256) k_grad_reduce(const float* __restrict__ gpart, int nb, float* __restrict__ grad) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kMlpParams) return;
    double a = 0.0;
#pragma unroll 8
    for (int b = 0; b < nb; ++b) a += gpart[(size_t)b * kMlpParams + p];  // block order; loads run ahead
    grad[p] = (float)a;
}

// Adam (Kingma and Ba 2015), step counted from 1.
__global__ void __launch_bounds__(256) k_adam(float* __restrict__ params, float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ grad, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kMlpParams) return;
    const float g = grad[p];
    const float mm = b1 * m[p] + (1.f - b1) * g;
    const float vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    params[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

}  // namespace gf

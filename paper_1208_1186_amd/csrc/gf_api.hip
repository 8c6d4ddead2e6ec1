// libgf host side: the C ABI declared in include/gf.h.
//
// The context carves the caller's workspace into: a device control block
// (theta, F, stop flag, iteration count, history), per-block reduction
// partials, FFT twiddle and sin^2 tables, the divergence buffer D, the FFT
// buffer Q, the gauge rows G and two link buffers (the loop kernel reads one
// and writes the other: after k updates the links are in buffer k & 1).
// Every kernel is queued on the caller's stream; the loop reads the control
// block back every check_every iterations, and kernels queued after the stop
// flag is set return at once, so the iterate is exactly the one the stopping
// rule selects.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/gf.h"
#include "gf_fft_ct.hpp"
#include "gf_kernels.hpp"

using namespace gf;

namespace {

constexpr int kEPT = 8;          // FFT elements held per thread per stage
constexpr int kMaxExtent = 64;   // largest supported extent
constexpr size_t kAlign = 256;
constexpr size_t kLdsMax = 160 * 1024;
constexpr int kPlanePad = 256;   // extra elements per plane: staggers plane starts across HBM channels

thread_local std::string g_init_error;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
int round64(int x) { return (x + 63) / 64 * 64; }

bool is_2a3b(int n) {
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

// Radix sequence for a length-n transform: threes first, then eights and fours, a two if left.
FftPlan make_plan(int n) {
    FftPlan p{};
    p.n = n;
    int m = n;
    while (m % 3 == 0) {
        p.rad[p.nst++] = 3;
        m /= 3;
    }
    int a = 0;
    while (m % 2 == 0) {
        ++a;
        m /= 2;
    }
    while (a >= 3 && a != 4) {
        p.rad[p.nst++] = 8;
        a -= 3;
    }
    while (a >= 2) {
        p.rad[p.nst++] = 4;
        a -= 2;
    }
    if (a == 1) p.rad[p.nst++] = 2;
    return p;
}

struct Layout {
    int n[4];
    int64_t vol;
    size_t ps;        // plane stride (elements) of every SoA array
    int nblk;         // blocks of the one-site-per-thread kernels
    int nblk_fused;   // blocks of the loop kernel (kFusedSites sites each)
    bool fp32;
    int ne;           // 9 or 6 complex entries stored per link
    // forward / inverse (x, y) pass over single-field planes
    int G, rs, thrA;
    size_t ldsA;
    // (z, t) pass
    int bx, tsp, thrB;
    size_t ldsB;
    // inverse (x, y) pass of four fields + gauge rows
    int thrC, eptC;
    size_t ldsC;
    // workspace offsets
    size_t off_ctl, off_part, off_sin2, off_tw, off_d, off_q, off_g, off_links[2], total;
};

gf_status plan_layout(const gf_params* p, Layout& L, std::string& err) {
    if (!p) {
        err = "params is NULL";
        return GF_EINVAL;
    }
    int64_t vol = 1;
    for (int i = 0; i < 4; ++i) {
        const int n = p->dims[i];
        if (n < 2) {
            err = "every extent must be >= 2";
            return GF_EINVAL;
        }
        if (n % 2 != 0 || !is_2a3b(n) || n > kMaxExtent) {
            err = "extent " + std::to_string(n) + " unsupported: each extent must be even, of the form 2^a 3^b and <= " +
                  std::to_string(kMaxExtent);
            return GF_ENOTSUP;
        }
        L.n[i] = n;
        vol *= n;
    }
    if (p->precision < GF_FP64_18 || p->precision > GF_MIXED) {
        err = "unknown precision";
        return GF_EINVAL;
    }
    if (p->precision == GF_MIXED) {
        err = "GF_MIXED is not available in this build";
        return GF_ENOTSUP;
    }
    if (!(p->alpha > 0.0) || !std::isfinite(p->alpha)) {
        err = "alpha must be positive and finite";
        return GF_EINVAL;
    }
    if (p->check_every < 1) {
        err = "check_every must be >= 1";
        return GF_EINVAL;
    }
    L.vol = vol;
    L.fp32 = p->precision == GF_FP32_12 || p->precision == GF_FP32_18;
    L.ne = (p->precision == GF_FP64_12 || p->precision == GF_FP32_12) ? 6 : 9;
    const size_t csz = L.fp32 ? 8 : 16;
    L.ps = align_up((size_t)vol, 256) + kPlanePad;
    L.nblk = (int)((vol + kSiteThreads - 1) / kSiteThreads);
    L.nblk_fused = (int)((vol + kFusedSites - 1) / kFusedSites);
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2], nt = L.n[3];
    // (x, y) pass: G planes per block, enough work per block, never straddling a field.
    const int nzt = nz * nt;
    L.G = 1;
    while (L.G * 2 <= nzt && nzt % (L.G * 2) == 0 && L.G * nx * ny < 512) L.G *= 2;
    L.rs = nx + 1;
    const int EA = L.G * nx * ny;
    L.thrA = std::min(1024, std::max(64, round64((EA + kEPT - 1) / kEPT)));
    L.ldsA = (size_t)(nx + ny) * csz + (size_t)L.G * ny * L.rs * csz;
    // (z, t) pass: bx consecutive x columns, up to 128 contiguous bytes per row.
    L.bx = 0;
    for (int b : {16, 8, 4, 2, 1}) {
        if (nx % b != 0) continue;
        const int E = b * nz * nt;
        const size_t lds = (size_t)(nz + nt) * csz + (size_t)nt * (nz * b + 1) * csz;
        if (E <= kEPT * 1024 && lds <= 80 * 1024 && (size_t)b * csz <= 128) {
            L.bx = b;
            break;
        }
    }
    if (L.bx == 0) {
        err = "z-t plane too large for one block";
        return GF_ENOTSUP;
    }
    L.tsp = nz * L.bx + 1;
    const int EB = L.bx * nz * nt;
    L.thrB = std::min(1024, std::max(64, round64((EB + kEPT - 1) / kEPT)));
    L.ldsB = (size_t)(nz + nt) * csz + (size_t)nt * L.tsp * csz;
    // inverse (x, y) + gauge pass: the four fields of one (z, t) plane per block.
    const int EC = 4 * nx * ny;
    L.eptC = EC <= kEPT * 1024 ? kEPT : 16;
    L.ldsC = (size_t)(nx + ny) * csz + (size_t)4 * ny * L.rs * csz;
    if (EC > L.eptC * (L.eptC == 16 ? 640 : 1024) || L.ldsC > kLdsMax) {
        err = "x-y plane too large for one block at this precision";
        return GF_ENOTSUP;
    }
    L.thrC = std::min(1024, std::max(64, round64((EC + L.eptC - 1) / L.eptC)));
    // Workspace.
    size_t o = 0;
    L.off_ctl = o;
    o = align_up(o + sizeof(Ctl), kAlign);
    L.off_part = o;
    o = align_up(o + (size_t)std::max(L.nblk, L.nblk_fused) * sizeof(double2), kAlign);
    L.off_sin2 = o;
    o = align_up(o + 4 * kMaxExtent * sizeof(double), kAlign);
    L.off_tw = o;
    o = align_up(o + 4 * kMaxExtent * 16, kAlign);
    L.off_d = o;
    o = align_up(o + 4 * L.ps * csz, kAlign);
    L.off_q = o;
    o = align_up(o + 4 * L.ps * csz, kAlign);
    L.off_g = o;
    o = align_up(o + 6 * L.ps * csz, kAlign);
    for (int i = 0; i < 2; ++i) {
        L.off_links[i] = o;
        o = align_up(o + (size_t)4 * L.ne * L.ps * csz, kAlign);
    }
    L.total = o;
    return GF_OK;
}

}  // namespace

struct gf_ctx {
    gf_params p;
    Layout L;
    Geom geom;
    hipStream_t st;
    double* links_user;
    unsigned char* ws;
    Ctl* ctl;
    double2* part;
    void* sin2;
    void* tw[4];
    void* D;      // divergence of the current links (four packed fields)
    void* Q;      // FFT work buffer (four packed fields)
    void* Gb;     // gauge rows (six planes)
    void* Lb[2];  // links after k updates live in Lb[k & 1]
    long long k_host;  // updates applied, as of the last read of the control block
    FftPlan plan[4];
    Ctl* h_head;  // pinned host copy of the control block's leading scalars
    std::string err;
    // Optional per-kernel HIP-event timing (gf_set_timing / gf_kernel_times).
    bool timing = false;
    std::vector<hipEvent_t> ev;  // 2 per pending measurement
    std::vector<int> ev_kid;
    int npend = 0;
    double kt_ms[GF_NKERNELS] = {};
    long long kt_n[GF_NKERNELS] = {};
};

namespace {

constexpr size_t kHeadBytes = offsetof(Ctl, hist_theta);

gf_status fail(gf_ctx* c, gf_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

gf_status check_hip(gf_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return GF_OK;
    return fail(c, GF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define GF_TRY_HIP(c, call)                               \
    do {                                                  \
        gf_status _s = check_hip((c), (call), #call);     \
        if (_s != GF_OK) return _s;                       \
    } while (0)

// ---------------------------------------------------------------- timing
constexpr int kEventPairs = 4096;

void tdrain(gf_ctx* c) {
    for (int i = 0; i < c->npend; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]) == hipSuccess) {
            c->kt_ms[c->ev_kid[i]] += ms;
            c->kt_n[c->ev_kid[i]] += 1;
        }
    }
    c->npend = 0;
}

// Record a start event for kernel kid (no-op unless timing is on).
void tstart(gf_ctx* c, int kid) {
    if (!c->timing) return;
    if (c->ev.empty()) {
        c->ev.resize(2 * kEventPairs);
        c->ev_kid.resize(kEventPairs);
        for (auto& e : c->ev) (void)hipEventCreate(&e);
    }
    if (c->npend == kEventPairs) {
        (void)hipStreamSynchronize(c->st);
        tdrain(c);
    }
    c->ev_kid[c->npend] = kid;
    (void)hipEventRecord(c->ev[2 * c->npend], c->st);
}
void tstop(gf_ctx* c) {
    if (!c->timing) return;
    (void)hipEventRecord(c->ev[2 * c->npend + 1], c->st);
    ++c->npend;
}

// ---------------------------------------------------------------- launches
int cur(const gf_ctx* c) { return (int)(c->k_host & 1); }
double inv3v(const gf_ctx* c) { return 1.0 / (3.0 * (double)c->L.vol); }
double inv12v(const gf_ctx* c) { return 1.0 / (12.0 * (double)c->L.vol); }

template <typename T, int NE>
Links<T, NE> links_of(gf_ctx* c, int i) {
    return Links<T, NE>{reinterpret_cast<cx<T>*>(c->Lb[i & 1]), c->L.ps};
}
template <typename T>
cx<T>* cxp(void* p) {
    return reinterpret_cast<cx<T>*>(p);
}
template <typename T>
const cx<T>* twp(gf_ctx* c, int d) {
    return reinterpret_cast<const cx<T>*>(c->tw[d]);
}

// Shapes with compile-time FFT kernels: (Nx, Ny, G) for the (x, y) passes,
// (Nz, Nt, bx) for the (z, t) pass at each precision, (Nx, Ny) for the gauge pass.
#define GF_XY_CASES(X) X(8, 8, 8) X(12, 12, 4) X(16, 16, 2) X(24, 24, 1) X(32, 32, 1) X(48, 48, 1)
#define GF_ZT_CASES_F64(X) \
    X(8, 8, 8) X(12, 12, 4) X(16, 16, 8) X(24, 8, 8) X(32, 4, 8) X(48, 8, 8) X(32, 32, 4) X(32, 64, 2)
#define GF_ZT_CASES_F32(X) \
    X(8, 8, 8) X(12, 12, 4) X(16, 16, 16) X(24, 8, 8) X(32, 4, 16) X(48, 8, 16) X(32, 32, 8) X(32, 64, 4)
#define GF_GAUGE_CASES(X) X(8, 8) X(12, 12) X(16, 16) X(24, 24) X(32, 32) X(48, 48)

bool generic_fft(const gf_ctx* c) { return (c->p.flags & GF_FLAG_GENERIC_FFT) != 0; }

template <typename T, bool INV>
bool launch_xy_ct(gf_ctx* c, const void* src, void* dst, int force, bool loop_reduce) {
    const Layout& L = c->L;
    const int nzt = L.n[2] * L.n[3];
    const cx<T>* s = reinterpret_cast<const cx<T>*>(src);
    const double2* part = loop_reduce ? c->part : nullptr;
#define GF_X(A, B, GG)                                                                                          \
    if (L.n[0] == A && L.n[1] == B && L.G == GG) {                                                              \
        hipLaunchKernelGGL((k_fft_xy_ct<T, A, B, GG, INV>), dim3(4 * nzt / GG), dim3(ct_threads(GG * A * B, 8)), \
                           0, c->st, s, cxp<T>(dst), L.ps, nzt, twp<T>(c, 0), twp<T>(c, 1), c->ctl, force, part,  \
                           L.nblk_fused, inv3v(c), inv12v(c));                                                  \
        return true;                                                                                            \
    }
    GF_XY_CASES(GF_X)
#undef GF_X
    return false;
}

template <typename T>
bool launch_zt_ct(gf_ctx* c, void* Z, T coef, int no_fa, int force) {
    const Layout& L = c->L;
    const T* s2 = reinterpret_cast<const T*>(c->sin2);
#define GF_X(A, B, BB)                                                                                     \
    if (L.n[2] == A && L.n[3] == B && L.bx == BB) {                                                        \
        hipLaunchKernelGGL((k_fft_zt_ct<T, A, B, BB>), dim3(4 * L.n[1] * (L.n[0] / BB)),                   \
                           dim3(ct_threads(BB * A * B, 8)), 0, c->st, cxp<T>(Z), L.ps, L.n[0], L.n[1],     \
                           twp<T>(c, 2), twp<T>(c, 3), s2, coef, no_fa, c->ctl, force);                    \
        return true;                                                                                       \
    }
    if constexpr (sizeof(T) == 8) {
        GF_ZT_CASES_F64(GF_X)
    } else {
        GF_ZT_CASES_F32(GF_X)
    }
#undef GF_X
    return false;
}

template <typename T>
bool launch_gauge_ct(gf_ctx* c, int force) {
    const Layout& L = c->L;
#define GF_X(A, B)                                                                                             \
    if (L.n[0] == A && L.n[1] == B) {                                                                          \
        hipLaunchKernelGGL((k_fft_xy_gauge_ct<T, A, B>), dim3(L.n[2] * L.n[3]),                                \
                           dim3(ct_threads(4 * A * B, gauge_ept(A, B))), gauge_ct_lds(A, B, sizeof(cx<T>)),    \
                           c->st, reinterpret_cast<const cx<T>*>(c->Q), L.ps, cxp<T>(c->Gb), L.ps,             \
                           twp<T>(c, 0), twp<T>(c, 1), c->ctl, force);                                         \
        return true;                                                                                           \
    }
    GF_GAUGE_CASES(GF_X)
#undef GF_X
    return false;
}

template <typename T>
void raise_lds_ct() {
#define GF_X(A, B)                                                                                     \
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_xy_gauge_ct<T, A, B>),            \
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
    GF_GAUGE_CASES(GF_X)
#undef GF_X
}

// (x, y) pass src -> dst. With loop_reduce, block 0 also reduces pending loop partials.
template <typename T, bool INV>
void launch_xy(gf_ctx* c, const void* src, void* dst, int force, bool loop_reduce) {
    const Layout& L = c->L;
    const int nzt = L.n[2] * L.n[3];
    tstart(c, INV ? GF_K_FFT_XY_INV : GF_K_FFT_XY_FWD);
    if (!generic_fft(c) && launch_xy_ct<T, INV>(c, src, dst, force, loop_reduce)) {
        tstop(c);
        return;
    }
    hipLaunchKernelGGL((k_fft_xy<T, kEPT, INV>), dim3(4 * nzt / L.G), dim3(L.thrA), L.ldsA, c->st,
                       reinterpret_cast<const cx<T>*>(src), cxp<T>(dst), L.ps, L.n[0], L.n[1], nzt, L.G, L.rs,
                       c->plan[0], c->plan[1], twp<T>(c, 0), twp<T>(c, 1), c->ctl, force,
                       loop_reduce ? c->part : nullptr, L.nblk_fused, inv3v(c), inv12v(c));
    tstop(c);
}

template <typename T>
void launch_zt(gf_ctx* c, void* Z, int force) {
    const Layout& L = c->L;
    const bool no_fa = (c->p.flags & GF_FLAG_NO_FA) != 0;
    const double coef = 0.5 * c->p.alpha * (no_fa ? 1.0 : 16.0) / (double)L.vol;
    tstart(c, GF_K_FFT_ZT);
    if (!generic_fft(c) && launch_zt_ct<T>(c, Z, (T)coef, no_fa ? 1 : 0, force)) {
        tstop(c);
        return;
    }
    hipLaunchKernelGGL((k_fft_zt<T, kEPT>), dim3(4 * L.n[1] * (L.n[0] / L.bx)), dim3(L.thrB), L.ldsB, c->st,
                       cxp<T>(Z), L.ps, L.n[0], L.n[1], L.n[2], L.n[3], L.bx, L.tsp, c->plan[2], c->plan[3],
                       twp<T>(c, 2), twp<T>(c, 3), reinterpret_cast<const T*>(c->sin2), (T)coef, no_fa ? 1 : 0,
                       c->ctl, force);
    tstop(c);
}

template <typename T>
void launch_gauge_pass(gf_ctx* c, int force) {
    const Layout& L = c->L;
    tstart(c, GF_K_FFT_XY_INV);
    if (!generic_fft(c) && launch_gauge_ct<T>(c, force)) {
        tstop(c);
        return;
    }
    if (L.eptC == kEPT)
        hipLaunchKernelGGL((k_fft_xy_gauge<T, kEPT>), dim3(L.n[2] * L.n[3]), dim3(L.thrC), L.ldsC, c->st,
                           reinterpret_cast<const cx<T>*>(c->Q), L.ps, cxp<T>(c->Gb), L.ps, L.n[0], L.n[1], L.rs,
                           c->plan[0], c->plan[1], twp<T>(c, 0), twp<T>(c, 1), c->ctl, force);
    else
        hipLaunchKernelGGL((k_fft_xy_gauge<T, 16>), dim3(L.n[2] * L.n[3]), dim3(L.thrC), L.ldsC, c->st,
                           reinterpret_cast<const cx<T>*>(c->Q), L.ps, cxp<T>(c->Gb), L.ps, L.n[0], L.n[1], L.rs,
                           c->plan[0], c->plan[1], twp<T>(c, 0), twp<T>(c, 1), c->ctl, force);
    tstop(c);
}

// Standalone measurement of the current links: Delta -> D, theta and F.
template <typename T, int NE>
void launch_measure_t(gf_ctx* c) {
    const Layout& L = c->L;
    tstart(c, GF_K_DIVERGENCE);
    hipLaunchKernelGGL((k_divergence<T, NE>), dim3(L.nblk), dim3(kSiteThreads), 0, c->st, links_of<T, NE>(c, cur(c)),
                       cxp<T>(c->D), L.ps, c->geom, c->part);
    tstop(c);
    tstart(c, GF_K_FINALIZE);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, c->st, c->part, L.nblk, inv3v(c), inv12v(c), c->ctl, 0);
    tstop(c);
}

// In-place update of the current links from (alpha/2) Delta~ packed in Q.
template <typename T, int NE>
void launch_update_t(gf_ctx* c) {
    const Layout& L = c->L;
    tstart(c, GF_K_UPDATE);
    hipLaunchKernelGGL((k_update<T, NE>), dim3(L.nblk), dim3(kSiteThreads), 0, c->st, links_of<T, NE>(c, cur(c)),
                       reinterpret_cast<const cx<T>*>(c->Q), L.ps, c->geom);
    tstop(c);
}

// Loop kernel from k to k + 1 updates: links Lb[k] -> Lb[k+1], divergence -> D.
template <typename T, int NE>
void launch_fused_t(gf_ctx* c, long long k) {
    const Layout& L = c->L;
    const int a = (int)(k & 1);
    tstart(c, GF_K_UPDATE_MEASURE);
    hipLaunchKernelGGL((k_update_measure<T, NE>), dim3(L.nblk_fused), dim3(kFusedThreads), 0, c->st,
                       links_of<T, NE>(c, a), links_of<T, NE>(c, 1 - a), reinterpret_cast<const cx<T>*>(c->Gb),
                       cxp<T>(c->D), L.ps, c->geom, c->part, c->ctl);
    tstop(c);
}

template <typename T, int NE>
void launch_pack_t(gf_ctx* c, const double* src) {
    hipLaunchKernelGGL((k_pack<T, NE>), dim3(c->L.nblk), dim3(kSiteThreads), 0, c->st, src,
                       links_of<T, NE>(c, cur(c)), c->L.vol, sizeof(T) == 4 ? 1 : 0);
}
template <typename T, int NE>
void launch_unpack_t(gf_ctx* c, double* dst) {
    hipLaunchKernelGGL((k_unpack<T, NE>), dim3(c->L.nblk), dim3(kSiteThreads), 0, c->st, links_of<T, NE>(c, cur(c)),
                       dst, c->L.vol);
}

#define GF_DISPATCH(c, fn, ...)                                                                  \
    do {                                                                                         \
        if ((c)->L.fp32) {                                                                       \
            if ((c)->L.ne == 6) fn<float, 6>(__VA_ARGS__); else fn<float, 9>(__VA_ARGS__);       \
        } else {                                                                                 \
            if ((c)->L.ne == 6) fn<double, 6>(__VA_ARGS__); else fn<double, 9>(__VA_ARGS__);     \
        }                                                                                        \
    } while (0)

gf_status launched(gf_ctx* c, const char* what) { return check_hip(c, hipGetLastError(), what); }

gf_status launch_measure(gf_ctx* c) {
    GF_DISPATCH(c, launch_measure_t, c);
    return launched(c, "divergence launch");
}

// Queue the update from k to k + 1 (no-ops on the device once the stop flag is set).
gf_status one_iteration(gf_ctx* c, long long k) {
    if (c->L.fp32) {
        launch_xy<float, false>(c, c->D, c->Q, 0, true);
        launch_zt<float>(c, c->Q, 0);
        launch_gauge_pass<float>(c, 0);
    } else {
        launch_xy<double, false>(c, c->D, c->Q, 0, true);
        launch_zt<double>(c, c->Q, 0);
        launch_gauge_pass<double>(c, 0);
    }
    GF_DISPATCH(c, launch_fused_t, c, k);
    return launched(c, "loop launch");
}

gf_status loop_finalize(gf_ctx* c) {
    tstart(c, GF_K_FINALIZE);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, c->st, c->part, c->L.nblk_fused, inv3v(c), inv12v(c),
                       c->ctl, 1);
    tstop(c);
    return launched(c, "finalize launch");
}

gf_status read_head(gf_ctx* c) {
    GF_TRY_HIP(c, hipMemcpyAsync(c->h_head, c->ctl, kHeadBytes, hipMemcpyDeviceToHost, c->st));
    GF_TRY_HIP(c, hipStreamSynchronize(c->st));
    if (c->npend) tdrain(c);
    c->k_host = c->h_head->iters;
    return GF_OK;
}

gf_status set_tol(gf_ctx* c, double tol) {
    hipLaunchKernelGGL(k_set_tol, dim3(1), dim3(64), 0, c->st, c->ctl, tol);
    return launched(c, "set_tol launch");
}

gf_status unpack_links(gf_ctx* c, double* dst) {
    GF_DISPATCH(c, launch_unpack_t, c, dst);
    return launched(c, "unpack launch");
}

// FFT kernels take more than 64 KB of dynamic LDS on large planes (gfx950 has 160 KB per CU).
void raise_lds_limits() {
    static bool done = false;
    if (done) return;
    const int cap = (int)kLdsMax;
    const void* fns[] = {
        reinterpret_cast<const void*>(&k_fft_xy<double, kEPT, false>),
        reinterpret_cast<const void*>(&k_fft_xy<double, kEPT, true>),
        reinterpret_cast<const void*>(&k_fft_zt<double, kEPT>),
        reinterpret_cast<const void*>(&k_fft_xy_gauge<double, kEPT>),
        reinterpret_cast<const void*>(&k_fft_xy_gauge<double, 16>),
        reinterpret_cast<const void*>(&k_fft_xy<float, kEPT, false>),
        reinterpret_cast<const void*>(&k_fft_xy<float, kEPT, true>),
        reinterpret_cast<const void*>(&k_fft_zt<float, kEPT>),
        reinterpret_cast<const void*>(&k_fft_xy_gauge<float, kEPT>),
        reinterpret_cast<const void*>(&k_fft_xy_gauge<float, 16>),
    };
    for (const void* f : fns) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    raise_lds_ct<double>();
    raise_lds_ct<float>();
    (void)hipGetLastError();
    done = true;
}

// sin^2 table [Nx | Ny | Nz | Nt] of 4 sin^2(pi n / N), then twiddles W_N^k per axis.
template <typename T>
void fill_tables(gf_ctx* c, std::vector<unsigned char>& host) {
    const Layout& L = c->L;
    const long double pi = 3.14159265358979323846264338327950288L;
    host.assign(L.off_d - L.off_sin2, 0);
    T* s2 = reinterpret_cast<T*>(host.data());
    int k = 0;
    for (int d = 0; d < 4; ++d)
        for (int n = 0; n < L.n[d]; ++n) {
            const long double sv = sinl(pi * (long double)n / (long double)L.n[d]);
            s2[k++] = (T)(4.0L * sv * sv);
        }
    for (int d = 0; d < 4; ++d) {
        cx<T>* tw = reinterpret_cast<cx<T>*>(host.data() + (L.off_tw - L.off_sin2) + (size_t)d * kMaxExtent * 16);
        for (int n = 0; n < L.n[d]; ++n) {
            const long double a = -2.0L * pi * (long double)n / (long double)L.n[d];
            tw[n] = {(T)cosl(a), (T)sinl(a)};
        }
    }
}

template <typename T>
void field_pack(gf_ctx* c, const void* src, void* dst) {
    hipLaunchKernelGGL(k_field_pack<T>, dim3(c->L.nblk), dim3(kSiteThreads), 0, c->st,
                       reinterpret_cast<const double*>(src), cxp<T>(dst), c->L.ps, c->L.vol, 1.0);
}
template <typename T>
void field_unpack(gf_ctx* c, const void* src, void* dst) {
    hipLaunchKernelGGL(k_field_unpack<T>, dim3(c->L.nblk), dim3(kSiteThreads), 0, c->st,
                       reinterpret_cast<const cx<T>*>(src), c->L.ps, reinterpret_cast<double*>(dst), c->L.vol);
}
template <typename T>
void gauge_unpack(gf_ctx* c, void* dst) {
    hipLaunchKernelGGL(k_gauge_unpack<T>, dim3(c->L.nblk), dim3(kSiteThreads), 0, c->st,
                       reinterpret_cast<const cx<T>*>(c->Gb), c->L.ps, reinterpret_cast<double*>(dst), c->L.vol);
}

// Forward FFT of Q, filter, and either the plain inverse (x, y) pass (gauge = false) or the gauge pass.
template <typename T>
void stage_spectral(gf_ctx* c, bool gauge) {
    launch_xy<T, false>(c, c->Q, c->Q, 1, false);
    launch_zt<T>(c, c->Q, 1);
    if (gauge)
        launch_gauge_pass<T>(c, 1);
    else
        launch_xy<T, true>(c, c->Q, c->Q, 1, false);
}

gf_status run_loop(gf_ctx* c, double tol, int64_t max_iter, gf_result* r) {
    const auto t0 = std::chrono::steady_clock::now();
    gf_status s = set_tol(c, tol);
    if (s == GF_OK) s = read_head(c);
    if (s != GF_OK) return s;
    const long long start = c->h_head->iters;
    while (!c->h_head->done && c->h_head->iters - start < max_iter) {
        const int64_t left = max_iter - (c->h_head->iters - start);
        const int64_t k = std::min<int64_t>(left, c->p.check_every);
        for (int64_t i = 0; i < k && s == GF_OK; ++i) s = one_iteration(c, c->k_host + i);
        if (s == GF_OK) s = loop_finalize(c);
        if (s == GF_OK) s = read_head(c);
        if (s != GF_OK) return s;
    }
    s = unpack_links(c, c->links_user);
    if (s == GF_OK) s = check_hip(c, hipStreamSynchronize(c->st), "sync");
    if (s != GF_OK) return s;
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (r) {
        r->iters = c->h_head->iters;
        r->theta = c->h_head->theta;
        r->F = c->h_head->F;
        r->phase = 1;
        r->fallbacks = 0;
        r->seconds = secs;
    }
    if (c->h_head->numeric) return fail(c, GF_ENUMERIC, "theta is not finite");
    return GF_OK;
}

}  // namespace

extern "C" {

size_t gf_workspace_bytes(const gf_params* params) {
    Layout L;
    std::string err;
    if (plan_layout(params, L, err) != GF_OK) return 0;
    return L.total;
}

gf_status gf_init(gf_ctx** out, const gf_params* params, void* d_links, void* d_workspace, size_t workspace_bytes,
                  void* stream) {
    try {
        if (!out) {
            g_init_error = "ctx output pointer is NULL";
            return GF_EINVAL;
        }
        *out = nullptr;
        Layout L;
        std::string err;
        gf_status s = plan_layout(params, L, err);
        if (s != GF_OK) {
            g_init_error = err;
            return s;
        }
        if (!d_links || !d_workspace) {
            g_init_error = "links or workspace pointer is NULL";
            return GF_EINVAL;
        }
        if (workspace_bytes < L.total) {
            g_init_error = "workspace too small: need " + std::to_string(L.total) + " bytes";
            return GF_EINVAL;
        }
        if ((reinterpret_cast<uintptr_t>(d_workspace) % kAlign) != 0) {
            g_init_error = "workspace must be 256-byte aligned";
            return GF_EINVAL;
        }
        gf_ctx* c = new (std::nothrow) gf_ctx();
        if (!c) {
            g_init_error = "out of host memory";
            return GF_EINVAL;
        }
        c->p = *params;
        c->L = L;
        c->st = reinterpret_cast<hipStream_t>(stream);
        c->links_user = reinterpret_cast<double*>(d_links);
        c->ws = reinterpret_cast<unsigned char*>(d_workspace);
        c->ctl = reinterpret_cast<Ctl*>(c->ws + L.off_ctl);
        c->part = reinterpret_cast<double2*>(c->ws + L.off_part);
        c->sin2 = c->ws + L.off_sin2;
        for (int d = 0; d < 4; ++d) c->tw[d] = c->ws + L.off_tw + (size_t)d * kMaxExtent * 16;
        c->D = c->ws + L.off_d;
        c->Q = c->ws + L.off_q;
        c->Gb = c->ws + L.off_g;
        for (int i = 0; i < 2; ++i) c->Lb[i] = c->ws + L.off_links[i];
        c->k_host = 0;
        for (int d = 0; d < 4; ++d) {
            c->geom.n[d] = L.n[d];
            c->plan[d] = make_plan(L.n[d]);
        }
        c->geom.vol = L.vol;
        c->geom.stride[0] = 1;
        for (int d = 1; d < 4; ++d) c->geom.stride[d] = c->geom.stride[d - 1] * L.n[d - 1];
        if (hipHostMalloc(reinterpret_cast<void**>(&c->h_head), kHeadBytes) != hipSuccess) {
            g_init_error = "hipHostMalloc of the control readback buffer failed";
            delete c;
            return GF_EDEVICE;
        }
        raise_lds_limits();
        std::vector<unsigned char> host;
        if (L.fp32)
            fill_tables<float>(c, host);
        else
            fill_tables<double>(c, host);
        Ctl head{};
        head.tol = -1.0;
        auto init_fail = [&](gf_status st) {
            g_init_error = c->err;
            (void)hipStreamSynchronize(c->st);
            (void)hipHostFree(c->h_head);
            delete c;
            return st;
        };
        if ((s = check_hip(c, hipMemcpyAsync(c->sin2, host.data(), host.size(), hipMemcpyHostToDevice, c->st),
                           "table upload")) != GF_OK)
            return init_fail(s);
        if ((s = check_hip(c, hipMemcpyAsync(c->ctl, &head, kHeadBytes, hipMemcpyHostToDevice, c->st),
                           "control upload")) != GF_OK)
            return init_fail(s);
        GF_DISPATCH(c, launch_pack_t, c, c->links_user);
        s = launched(c, "pack launch");
        if (s == GF_OK) s = launch_measure(c);
        if (s == GF_OK) s = read_head(c);
        if (s != GF_OK) return init_fail(s);
        *out = c;
        return GF_OK;
    } catch (...) {
        g_init_error = "unexpected host exception";
        return GF_EINVAL;
    }
}

gf_status gf_iterate(gf_ctx* c, int64_t n, gf_result* r) {
    if (!c) return GF_EINVAL;
    if (n < 0) return fail(c, GF_EINVAL, "n must be >= 0");
    try {
        return run_loop(c, -1.0, n, r);
    } catch (...) {
        return fail(c, GF_EINVAL, "unexpected host exception");
    }
}

gf_status gf_fix_until(gf_ctx* c, double tol, int64_t max_iter, gf_result* r) {
    if (!c) return GF_EINVAL;
    if (!(tol > 0.0)) return fail(c, GF_EINVAL, "theta_tol must be > 0");
    if (max_iter < 0) return fail(c, GF_EINVAL, "max_iter must be >= 0");
    try {
        gf_status s = run_loop(c, tol, max_iter, r);
        if (s != GF_OK) return s;
        if (!c->h_head->done) return fail(c, GF_ENOTCONV, "max_iter reached before theta < tol");
        return GF_OK;
    } catch (...) {
        return fail(c, GF_EINVAL, "unexpected host exception");
    }
}

gf_status gf_quality(gf_ctx* c, double* theta, double* F) {
    if (!c) return GF_EINVAL;
    if (!theta || !F) return fail(c, GF_EINVAL, "null output");
    gf_status s = read_head(c);
    if (s != GF_OK) return s;
    *theta = c->h_head->theta;
    *F = c->h_head->F;
    return GF_OK;
}

gf_status gf_get_links(gf_ctx* c, void* d_out) {
    if (!c) return GF_EINVAL;
    if (!d_out) return fail(c, GF_EINVAL, "d_out is NULL");
    gf_status s = unpack_links(c, reinterpret_cast<double*>(d_out));
    if (s != GF_OK) return s;
    return check_hip(c, hipStreamSynchronize(c->st), "sync");
}

gf_status gf_history(gf_ctx* c, int64_t n, double* h_theta, double* h_F) {
    if (!c) return GF_EINVAL;
    if (!h_theta || !h_F) return fail(c, GF_EINVAL, "null output");
    gf_status s = read_head(c);
    if (s != GF_OK) return s;
    const long long it = c->h_head->iters;
    if (n < 0 || n > kHist || n > it + 1) return fail(c, GF_EINVAL, "n out of range");
    std::vector<double> th(kHist), f(kHist);
    GF_TRY_HIP(c, hipMemcpyAsync(th.data(), c->ctl->hist_theta, kHist * sizeof(double), hipMemcpyDeviceToHost, c->st));
    GF_TRY_HIP(c, hipMemcpyAsync(f.data(), c->ctl->hist_F, kHist * sizeof(double), hipMemcpyDeviceToHost, c->st));
    GF_TRY_HIP(c, hipStreamSynchronize(c->st));
    for (int64_t i = 0; i < n; ++i) {
        const long long k = it - n + 1 + i;
        h_theta[i] = th[k % kHist];
        h_F[i] = f[k % kHist];
    }
    return GF_OK;
}

gf_status gf_stage_divergence(gf_ctx* c, void* d_delta) {
    if (!c) return GF_EINVAL;
    if (!d_delta) return fail(c, GF_EINVAL, "d_delta is NULL");
    gf_status s = launch_measure(c);
    if (s != GF_OK) return s;
    if (c->L.fp32)
        field_unpack<float>(c, c->D, d_delta);
    else
        field_unpack<double>(c, c->D, d_delta);
    s = launched(c, "field unpack launch");
    if (s != GF_OK) return s;
    return read_head(c);
}

gf_status gf_stage_filter(gf_ctx* c, const void* d_in, void* d_out) {
    if (!c) return GF_EINVAL;
    if (!d_in || !d_out) return fail(c, GF_EINVAL, "null pointer");
    if (c->L.fp32) {
        field_pack<float>(c, d_in, c->Q);
        stage_spectral<float>(c, false);
        field_unpack<float>(c, c->Q, d_out);
    } else {
        field_pack<double>(c, d_in, c->Q);
        stage_spectral<double>(c, false);
        field_unpack<double>(c, c->Q, d_out);
    }
    gf_status s = launched(c, "filter launch");
    if (s != GF_OK) return s;
    return check_hip(c, hipStreamSynchronize(c->st), "sync");
}

gf_status gf_stage_gauge(gf_ctx* c, const void* d_in, void* d_out) {
    if (!c) return GF_EINVAL;
    if (!d_in || !d_out) return fail(c, GF_EINVAL, "null pointer");
    if (c->L.fp32) {
        field_pack<float>(c, d_in, c->Q);
        stage_spectral<float>(c, true);
        gauge_unpack<float>(c, d_out);
    } else {
        field_pack<double>(c, d_in, c->Q);
        stage_spectral<double>(c, true);
        gauge_unpack<double>(c, d_out);
    }
    gf_status s = launched(c, "gauge launch");
    if (s != GF_OK) return s;
    return check_hip(c, hipStreamSynchronize(c->st), "sync");
}

gf_status gf_stage_update(gf_ctx* c, const void* d_scaled) {
    if (!c) return GF_EINVAL;
    if (!d_scaled) return fail(c, GF_EINVAL, "null pointer");
    if (c->L.fp32)
        field_pack<float>(c, d_scaled, c->Q);
    else
        field_pack<double>(c, d_scaled, c->Q);
    GF_DISPATCH(c, launch_update_t, c);
    gf_status s = launched(c, "update launch");
    if (s == GF_OK) s = unpack_links(c, c->links_user);
    if (s == GF_OK) s = launch_measure(c);  // theta, F and divergence of the updated links
    if (s != GF_OK) return s;
    return read_head(c);
}

gf_status gf_set_timing(gf_ctx* c, int32_t enable) {
    if (!c) return GF_EINVAL;
    GF_TRY_HIP(c, hipStreamSynchronize(c->st));
    tdrain(c);
    c->timing = enable != 0;
    for (int i = 0; i < GF_NKERNELS; ++i) {
        c->kt_ms[i] = 0.0;
        c->kt_n[i] = 0;
    }
    return GF_OK;
}

gf_status gf_kernel_times(gf_ctx* c, int32_t n, double* h_ms_total, int64_t* h_counts) {
    if (!c) return GF_EINVAL;
    if (!h_ms_total || !h_counts || n < 0 || n > GF_NKERNELS) return fail(c, GF_EINVAL, "bad arguments");
    GF_TRY_HIP(c, hipStreamSynchronize(c->st));
    tdrain(c);
    for (int i = 0; i < n; ++i) {
        h_ms_total[i] = c->kt_ms[i];
        h_counts[i] = c->kt_n[i];
    }
    return GF_OK;
}

const char* gf_last_error(const gf_ctx* c) { return c ? c->err.c_str() : g_init_error.c_str(); }

void gf_destroy(gf_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->st);
    if (c->h_head) (void)hipHostFree(c->h_head);
    for (auto& e : c->ev) (void)hipEventDestroy(e);
    delete c;
}

}  // extern "C"

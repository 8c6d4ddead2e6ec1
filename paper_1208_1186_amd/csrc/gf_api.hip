// libgf host side: the C ABI declared in include/gf.h.
//
// The context carves the caller's workspace into: a device control block
// (theta, F, stop flag, iteration count, history), per-block reduction
// partials, FFT twiddle and sin^2 tables, the divergence buffer D, the FFT
// buffer Q, the input links U0 (never written after gf_init) and two buffers
// of the accumulated gauge transform H (rows 1-2): after k updates the current
// links are H U0 H(x+mu)^dag with H in buffer k & 1 (the inverse (x, y) pass of
// update k reads buffer k & 1 and writes the other).
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
#include <map>
#include <mutex>
#include <vector>

#include "../../include/gf.h"
#include "gf_fft_ct.hpp"
#include "gf_fft_reg.hpp"
#include "gf_batch.hpp"
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
    int zb = 1;       // loop-kernel traversal: z planes per group inside the t loop, 0: blocks step
                      // through t, -1: bricks step through t segments (autotuned)
    BrickGeom bk{};   // brick march geometry (bk.by == 0: the shape has none)
    int bk_threads = 0;
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
    bool learned;     // reserve the network parameters and the multiplier table
    bool record;      // reserve two spectra and the per-tuple record
    int ntuples;      // distinct momentum tuples (N_mu/2 + 1 per axis)
    // workspace offsets
    size_t off_ctl, off_tune, off_part, off_sin2, off_tw, off_d, off_q, off_h[2], off_links, off_mlp, off_mtab,
        off_spec[4], off_rec, total;
    // GF_MIXED: a float child (bulk) and a double child (polish) share the workspace
    bool mixed;
    size_t child_off[2];
};

// Launch shape of the (x, y) passes for G planes per block, and of the (z, t)
// pass for bx columns per block.
void set_xy_tile(Layout& L, int G) {
    const size_t csz = L.fp32 ? 8 : 16;
    L.G = G;
    L.rs = L.n[0] + 1;
    L.thrA = std::min(1024, std::max(64, round64((G * L.n[0] * L.n[1] + kEPT - 1) / kEPT)));
    L.ldsA = (size_t)(L.n[0] + L.n[1]) * csz + (size_t)G * L.n[1] * L.rs * csz;
}
void set_zt_tile(Layout& L, int bx) {
    const size_t csz = L.fp32 ? 8 : 16;
    L.bx = bx;
    L.tsp = L.n[2] * bx + bx;  // consecutive lanes of a z stage in consecutive LDS slots (see k_fft_zt_ct)
    L.thrB = std::min(1024, std::max(64, round64((bx * L.n[2] * L.n[3] + kEPT - 1) / kEPT)));
    L.ldsB = (size_t)(L.n[2] + L.n[3]) * csz + (size_t)L.n[3] * L.tsp * csz;
}

// (z, t) planes whose pass holds whole lines in registers (k_fft_zt_reg, BX columns per block); for these
// shapes it replaces the LDS Stockham tilings. Measured at 32^4: float 23.9 against 32.1 us (21.0-21.2
// against 21.3-21.4 once the LDS stages read and wrote memory directly and shared the filter stage); in double the
// 32-point lines take all 256 registers (one wave per SIMD) and the pass was slower (47.7 against 43.6 us),
// as was float on 32 x 64 planes (103 against 71 us), so those keep the LDS passes.
#define GF_ZT_REG_F64(X)
#define GF_ZT_REG_F32(X) X(32, 32, 8)

// Columns per block of the register (z, t) pass of this shape, or 0 if the shape takes the LDS tilings.
int zt_reg_bx(const Layout& L) {
#define GF_X(A, B, BB) \
    if (L.n[2] == A && L.n[3] == B && L.n[0] % BB == 0) return BB;
    if (L.fp32) {
        GF_ZT_REG_F32(GF_X)
    } else {
        GF_ZT_REG_F64(GF_X)
    }
#undef GF_X
    return 0;
}

void plan_brick(Layout& L);

gf_status plan_plain(const gf_params* p, Layout& L, std::string& err) {
    if (!p) {
        err = "params is NULL";
        return GF_EINVAL;
    }
    L.mixed = false;
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
    if (!(p->alpha > 0.0) || !std::isfinite(p->alpha)) {
        err = "alpha must be positive and finite";
        return GF_EINVAL;
    }
    if (p->check_every < 1) {
        err = "check_every must be >= 1";
        return GF_EINVAL;
    }
    L.vol = vol;
    L.learned = (p->flags & GF_FLAG_LEARNED) != 0;
    L.record = (p->flags & GF_FLAG_RECORD_SPECTRA) != 0;
    L.ntuples = (L.n[0] / 2 + 1) * (L.n[1] / 2 + 1) * (L.n[2] / 2 + 1) * (L.n[3] / 2 + 1);
    L.fp32 = p->precision == GF_FP32_12 || p->precision == GF_FP32_18;
    L.ne = (p->precision == GF_FP64_12 || p->precision == GF_FP32_12) ? 6 : 9;
    const size_t csz = L.fp32 ? 8 : 16;
    L.ps = align_up((size_t)vol, 256) + kPlanePad;
    L.nblk = (int)((vol + kSiteThreads - 1) / kSiteThreads);
    L.nblk_fused = (int)((vol + kFusedSites - 1) / kFusedSites);
    plan_brick(L);
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2], nt = L.n[3];
    // (x, y) pass: G planes per block, enough work per block, never straddling a field.
    const int nzt = nz * nt;
    // (the default; gf_init times the compile-time alternatives of the shape and keeps the fastest)
    const int want = nx * ny >= 1024 ? 2048 : 512;
    int G = 1;
    while (G * 2 <= nzt && nzt % (G * 2) == 0 && G * nx * ny < want) G *= 2;
    set_xy_tile(L, G);
    // (z, t) pass: bx consecutive x columns, up to 128 contiguous bytes per row.
    L.bx = 0;
    for (int b : {16, 8, 4, 2, 1}) {
        if (nx % b != 0) continue;
        const int E = b * nz * nt;
        const size_t lds = (size_t)(nz + nt) * csz + (size_t)nt * (nz * b + b) * csz;
        if (E <= kEPT * 1024 && lds <= 80 * 1024 && (size_t)b * csz <= 128) {
            L.bx = b;
            break;
        }
    }
    if (L.bx == 0) {
        err = "z-t plane too large for one block";
        return GF_ENOTSUP;
    }
    if (const int rb = zt_reg_bx(L)) L.bx = rb;  // the register pass of this shape
    set_zt_tile(L, L.bx);
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
    L.off_tune = o;  // a scratch control-block head for the autotuner's trial launches of the loop kernel
    o = align_up(o + offsetof(Ctl, hist_theta), kAlign);
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
    for (int i = 0; i < 2; ++i) {
        L.off_h[i] = o;
        o = align_up(o + 6 * L.ps * csz, kAlign);
    }
    L.off_links = o;
    o = align_up(o + (size_t)4 * L.ne * L.ps * csz, kAlign);
    L.off_mlp = o;
    if (L.learned) o = align_up(o + kMlpParams * sizeof(float), kAlign);
    L.off_mtab = o;
    if (L.learned) o = align_up(o + (size_t)L.ntuples * csz / 2, kAlign);
    for (int i = 0; i < 4; ++i) {
        L.off_spec[i] = o;
        if (L.record) o = align_up(o + 4 * L.ps * csz, kAlign);
    }
    L.off_rec = o;
    if (L.record) o = align_up(o + (size_t)L.ntuples * 3 * sizeof(double), kAlign);
    L.total = o;
    return GF_OK;
}

// Parameters of the two children of a GF_MIXED context.
gf_params mixed_child(const gf_params& p, int which) {
    gf_params q = p;
    q.precision = which == 0 ? GF_FP32_12 : GF_FP64_18;
    q.flags |= GF_FLAG_ACCUMULATE_GAUGE;
    return q;
}

gf_status plan_layout(const gf_params* p, Layout& L, std::string& err) {
    if (p && p->precision == GF_MIXED) {
        if (!(p->switch_theta > 0.0) || !std::isfinite(p->switch_theta)) {
            err = "switch_theta must be positive and finite";
            return GF_EINVAL;
        }
        Layout a, b;
        gf_params q0 = mixed_child(*p, 0), q1 = mixed_child(*p, 1);
        gf_status s = plan_plain(&q0, a, err);
        if (s == GF_OK) s = plan_plain(&q1, b, err);
        if (s != GF_OK) return s;
        L = b;
        L.mixed = true;
        L.child_off[0] = 0;
        L.child_off[1] = align_up(a.total, kAlign);
        L.total = L.child_off[1] + b.total;
        return GF_OK;
    }
    return plan_plain(p, L, err);
}

struct BatchState;

}  // namespace

struct gf_ctx {
    gf_params p;
    Layout L;
    Geom geom;
    hipStream_t st;
    double* links_user;
    unsigned char* ws;
    Ctl* ctl;
    Ctl* tune_ctl;  // head only: the autotuner's trial launches of the loop kernel
    double2* part;
    void* sin2;
    void* tw[4];
    void* D;      // divergence of the current links (four packed fields)
    void* Q;      // FFT work buffer (four packed fields)
    void* U0;     // the input links (SoA planes)
    void* Hb[2];  // accumulated gauge transform rows after k updates in Hb[k & 1]
    // learned preconditioner state
    TupleGeom tg;
    float* mlp;          // network parameters (workspace copy)
    void* mtab;          // multiplier per tuple for the current iteration
    bool net_on = false;       // gf_mlp_set_weights called and not disabled
    bool net_this = false;     // the iteration being queued uses the table
    int rejects = 0;           // rejected learned steps since gf_mlp_set_weights
    long long net_pause = 0;   // plain updates still to take before the network is tried again
    int fallbacks = 0;         // rejected learned steps in total
    // spectrum recording
    void* spec[4];  // spectra of the plain iterates (0, 1) and of the probe steps (2, 3)
    double coef_scale = 1.0;  // factor on the plain multiplier (the recorder's probe step)
    double* rec;
    void* spec_capture = nullptr;  // where the (z, t) pass writes the spectrum, if anywhere
    // GF_MIXED parent: the float and double children, and the active phase
    gf_ctx* child[2] = {nullptr, nullptr};
    int phase = 1;
    long long k_host;  // updates applied, as of the last read of the control block
    // A batch driver launches the loop kernels over nact configurations at once
    // (blockIdx.y indexes act_dev); the buffers of configuration c are c*cs
    // bytes after this context's. Single lattices have nact 1, cs 0.
    int nact = 1;
    const int* act_dev = nullptr;
    size_t cs = 0;
    BatchState* batch = nullptr;  // set on a context made by gf_init_batch
    FftPlan plan[4];
    Ctl* h_head;  // pinned host copy of the control block's leading scalars
    bool own_head = true;  // h_head was allocated here (not a slot of a batch group's array)
    std::string err;
    // Optional per-kernel HIP-event timing (gf_set_timing / gf_kernel_times).
    bool timing = false;
    uint32_t timing_mask = 0;  // kernel ids (bit GF_K_*) timed while timing is on
    bool timing_now = false;   // the launch being queued is bracketed by events
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
    c->timing_now = c->timing && ((c->timing_mask >> kid) & 1u);
    if (!c->timing_now) return;
    if (c->ev.empty()) {
        c->ev.resize(2 * kEventPairs);
        c->ev_kid.resize(kEventPairs);
        // timing only: no system-scope fence (cache write-back) when an event completes, which would
        // slow the kernels that follow it
        for (auto& e : c->ev) (void)hipEventCreateWithFlags(&e, hipEventDisableSystemFence);
    }
    if (c->npend == kEventPairs) {
        (void)hipStreamSynchronize(c->st);
        tdrain(c);
    }
    c->ev_kid[c->npend] = kid;
    (void)hipEventRecord(c->ev[2 * c->npend], c->st);
}
void tstop(gf_ctx* c) {
    if (!c->timing_now) return;
    (void)hipEventRecord(c->ev[2 * c->npend + 1], c->st);
    ++c->npend;
}

// ---------------------------------------------------------------- launches
int cur(const gf_ctx* c) { return (int)(c->k_host & 1); }

// g = reunitarize(exp((alpha/2) Delta~)) instead of the first-order 1 + (alpha/2) Delta~.
int exact_exp(const gf_ctx* c) { return (c->p.flags & GF_FLAG_EXACT_EXP) ? 1 : 0; }
Batch bt(const gf_ctx* c) { return Batch{c->act_dev, c->cs}; }
double inv3v(const gf_ctx* c) { return 1.0 / (3.0 * (double)c->L.vol); }
double inv12v(const gf_ctx* c) { return 1.0 / (12.0 * (double)c->L.vol); }

template <typename T, int NE>
Links<T, NE> links_of(gf_ctx* c) {
    return Links<T, NE>{reinterpret_cast<cx<T>*>(c->U0), c->L.ps};
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
// Several entries per shape are the alternatives the autotuner times. 32 x 32 planes have no
// one-plane (x, y) tiling: timed on its own it came out fastest (23 against 29 us at 32^4 in double)
// and the autotuner kept it on most runs, but inside the loop, after the loop kernel, it took 31 us
// against 27 us for two planes per block (34.5-35 against 30-31 while one of its blocks also reduced
// the loop kernel's partials), whichever way the trials were ordered.
#define GF_XY_CASES(X)                                                                                         \
    X(8, 8, 8) X(8, 8, 16) X(8, 8, 32) X(12, 12, 4) X(12, 12, 8) X(12, 12, 16) X(16, 16, 2) X(16, 16, 4)       \
    X(16, 16, 8) X(24, 24, 1) X(24, 24, 2) X(24, 24, 4) X(32, 32, 2) X(32, 32, 4) X(48, 48, 1)                \
    X(48, 48, 2)
#define GF_ZT_CASES_F64(X)                                                                                     \
    X(8, 8, 4) X(8, 8, 8) X(12, 12, 2) X(12, 12, 4) X(16, 16, 4) X(16, 16, 8) X(16, 16, 16) X(24, 8, 4)        \
    X(24, 8, 8) X(32, 4, 4) X(32, 4, 8) X(32, 4, 16) X(48, 8, 2) X(48, 8, 4) X(48, 8, 8) X(48, 8, 16)         \
    X(32, 32, 2) X(32, 32, 4) X(32, 64, 2)
#define GF_ZT_CASES_F32(X)                                                                                     \
    X(8, 8, 4) X(8, 8, 8) X(12, 12, 4) X(16, 16, 4) X(16, 16, 8) X(16, 16, 16) X(24, 8, 4) X(24, 8, 8)        \
    X(32, 4, 8) X(32, 4, 16) X(32, 4, 32) X(48, 8, 4) X(48, 8, 8) X(48, 8, 16) X(32, 32, 4) X(32, 32, 8)      \
    X(32, 64, 2) X(32, 64, 4)
#define GF_GAUGE_CASES(X) X(8, 8) X(12, 12) X(16, 16) X(24, 24) X(32, 32) X(48, 48)

bool generic_fft(const gf_ctx* c) { return (c->p.flags & (GF_FLAG_GENERIC_FFT | GF_FLAG_BATCH_FUSED)) != 0; }

template <typename T, bool INV>
bool launch_xy_ct(gf_ctx* c, const void* src, void* dst, int force, bool loop_reduce) {
    const Layout& L = c->L;
    const int nzt = L.n[2] * L.n[3];
    const cx<T>* s = reinterpret_cast<const cx<T>*>(src);
    const double2* part = loop_reduce ? c->part : nullptr;
#define GF_X(A, B, GG)                                                                                          \
    if (L.n[0] == A && L.n[1] == B && L.G == GG) {                                                              \
        hipLaunchKernelGGL((k_fft_xy_ct<T, A, B, GG, INV>), dim3(4 * nzt / GG + (part ? 1 : 0), c->nact),         \
                           dim3(ct_threads(GG * A * B, 8)), 0, c->st, s, cxp<T>(dst), L.ps, nzt, twp<T>(c, 0),  \
                           twp<T>(c, 1), c->ctl, force, part, L.nblk_fused, inv3v(c), inv12v(c), bt(c));       \
        return true;                                                                                            \
    }
    GF_XY_CASES(GF_X)
#undef GF_X
    return false;
}


template <typename T>
bool launch_zt_ct(gf_ctx* c, void* Z, T coef, int no_fa, int force, const T* mtab, cx<T>* spec) {
    const Layout& L = c->L;
    const T* s2 = reinterpret_cast<const T*>(c->sin2);
#define GF_X(A, B, BB)                                                                                     \
    if (L.n[2] == A && L.n[3] == B && L.n[0] % BB == 0) {                                                  \
        hipLaunchKernelGGL((k_fft_zt_reg<T, A, B, BB>), dim3(4 * L.n[1] * (L.n[0] / BB), c->nact),          \
                           dim3(BB * (A > B ? A : B)), 0, c->st, cxp<T>(Z), L.ps, L.n[0], L.n[1],          \
                           twp<T>(c, 2), twp<T>(c, 3), s2, coef, no_fa, c->ctl, force, mtab, c->tg, spec,  \
                           bt(c));                                                                         \
        return true;                                                                                       \
    }
    if constexpr (sizeof(T) == 8) {
        GF_ZT_REG_F64(GF_X)
    } else {
        GF_ZT_REG_F32(GF_X)
    }
#undef GF_X
    if (L.n[0] > kZtMaxXY || L.n[1] > kZtMaxXY) return false;
#define GF_X(A, B, BB)                                                                                     \
    if (L.n[2] == A && L.n[3] == B && L.bx == BB) {                                                        \
        hipLaunchKernelGGL((k_fft_zt_ct<T, A, B, BB>), dim3(4 * L.n[1] * (L.n[0] / BB), c->nact),           \
                           dim3(ct_threads(BB * A * B, 8)), 0, c->st, cxp<T>(Z), L.ps, L.n[0], L.n[1],     \
                           twp<T>(c, 2), twp<T>(c, 3), s2, coef, no_fa, c->ctl, force, mtab, c->tg, spec,  \
                           bt(c));                                                                         \
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
bool launch_gauge_ct(gf_ctx* c, int force, const void* hin, void* hout) {
    const Layout& L = c->L;
#define GF_X(A, B)                                                                                             \
    if (L.n[0] == A && L.n[1] == B) {                                                                          \
        hipLaunchKernelGGL((k_fft_xy_gauge_ct<T, A, B>), dim3(L.n[2] * L.n[3], c->nact),                       \
                           dim3(ct_threads(4 * A * B, gauge_ept(A, B))), gauge_ct_lds(A, B, sizeof(cx<T>)),    \
                           c->st, reinterpret_cast<const cx<T>*>(c->Q), L.ps,                                  \
                           reinterpret_cast<const cx<T>*>(hin), cxp<T>(hout), twp<T>(c, 0), twp<T>(c, 1),       \
                           c->ctl, force, bt(c), exact_exp(c));                                                \
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
    hipLaunchKernelGGL((k_fft_xy<T, kEPT, INV>), dim3(4 * nzt / L.G + (loop_reduce ? 1 : 0), c->nact), dim3(L.thrA),
                       L.ldsA, c->st,
                       reinterpret_cast<const cx<T>*>(src), cxp<T>(dst), L.ps, L.n[0], L.n[1], nzt, L.G, L.rs,
                       c->plan[0], c->plan[1], twp<T>(c, 0), twp<T>(c, 1), c->ctl, force,
                       loop_reduce ? c->part : nullptr, L.nblk_fused, inv3v(c), inv12v(c), bt(c));
    tstop(c);
}

template <typename T>
void launch_zt(gf_ctx* c, void* Z, int force) {
    const Layout& L = c->L;
    const bool no_fa = (c->p.flags & GF_FLAG_NO_FA) != 0;
    const double coef = 0.5 * c->p.alpha * (no_fa ? 1.0 : 16.0) / (double)L.vol * c->coef_scale;
    tstart(c, GF_K_FFT_ZT);
    const T* mtab = c->net_this ? reinterpret_cast<const T*>(c->mtab) : nullptr;
    cx<T>* spec = reinterpret_cast<cx<T>*>(c->spec_capture);
    if (!generic_fft(c) && launch_zt_ct<T>(c, Z, (T)coef, no_fa ? 1 : 0, force, mtab, spec)) {
        tstop(c);
        return;
    }
    hipLaunchKernelGGL((k_fft_zt<T, kEPT>), dim3(4 * L.n[1] * (L.n[0] / L.bx), c->nact), dim3(L.thrB), L.ldsB,
                       c->st, cxp<T>(Z), L.ps, L.n[0], L.n[1], L.n[2], L.n[3], L.bx, L.tsp, c->plan[2], c->plan[3],
                       twp<T>(c, 2), twp<T>(c, 3), reinterpret_cast<const T*>(c->sin2), (T)coef, no_fa ? 1 : 0,
                       c->ctl, force, mtab, c->tg, spec, bt(c));
    tstop(c);
}

// Inverse (x, y) pass + gauge: hout = reunitarize(g hin) (hin null: g itself).
template <typename T>
void launch_gauge_pass(gf_ctx* c, int force, const void* hin, void* hout) {
    const Layout& L = c->L;
    tstart(c, GF_K_FFT_XY_INV);
    if (!generic_fft(c) && launch_gauge_ct<T>(c, force, hin, hout)) {
        tstop(c);
        return;
    }
    const cx<T>* hi = reinterpret_cast<const cx<T>*>(hin);
    if (L.eptC == kEPT)
        hipLaunchKernelGGL((k_fft_xy_gauge<T, kEPT>), dim3(L.n[2] * L.n[3], c->nact), dim3(L.thrC), L.ldsC, c->st,
                           reinterpret_cast<const cx<T>*>(c->Q), L.ps, hi, cxp<T>(hout), L.n[0], L.n[1], L.rs,
                           c->plan[0], c->plan[1], twp<T>(c, 0), twp<T>(c, 1), c->ctl, force, bt(c),
                           exact_exp(c));
    else
        hipLaunchKernelGGL((k_fft_xy_gauge<T, 16>), dim3(L.n[2] * L.n[3], c->nact), dim3(L.thrC), L.ldsC, c->st,
                           reinterpret_cast<const cx<T>*>(c->Q), L.ps, hi, cxp<T>(hout), L.n[0], L.n[1], L.rs,
                           c->plan[0], c->plan[1], twp<T>(c, 0), twp<T>(c, 1), c->ctl, force, bt(c),
                           exact_exp(c));
    tstop(c);
}

// Blocks of the loop kernel: one per site block, (t-march) one per 64-site run of the (x, y, z) volume,
// or (brick march) one per brick and t segment.
int loop_blocks(const Layout& L) {
    if (L.zb == -1) return L.bk.nby * L.bk.nbz * (L.n[3] / L.bk.lt);
    return L.zb == 0 ? (int)(L.vol / L.n[3] / kFusedSites) : L.nblk_fused;
}

// Brick march geometry of a shape, if it has one: rows in y the fewest that make Nx*by a multiple of 64,
// planes in z the most that keep a brick at 512 threads (1024 if one plane already needs more than 512),
// t segments short enough for 1024 blocks (at least 2 steps each).
void plan_brick(Layout& L) {
    L.bk = BrickGeom{};
    L.bk_threads = 0;
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2], nt = L.n[3];
    int by = 0;
    for (int d = 1; d <= ny; ++d)
        if (ny % d == 0 && (nx * d) % kFusedSites == 0) {
            by = d;
            break;
        }
    if (by == 0 || 4 * nx * by > 1024) return;
    const int cap = 4 * nx * by > 512 ? 1024 : 512;
    int bz = 1;
    for (int d = 1; d <= nz; ++d)
        if (nz % d == 0 && 4 * nx * by * d <= cap) bz = d;
    const int bricks = (ny / by) * (nz / bz);
    int lt = nt;
    for (int d = nt; d >= 2; --d)
        if (nt % d == 0) {
            lt = d;
            if (bricks * (nt / d) >= 1024) break;
        }
    if (lt < 2 || brick_lds(nx, ny, nz, by, bz, L.fp32 ? 4 : 8) > kLdsMax - 1024) return;
    // 32-bit byte offsets into the link planes (4 * NE planes) and the divergence planes
    if ((size_t)4 * L.ne * L.ps * (L.fp32 ? 8 : 16) >= ((size_t)1 << 32)) return;
    L.bk = BrickGeom{by, bz, ny / by, nz / bz, lt};
    L.bk_threads = 4 * nx * by * bz;
}

template <typename T, int NE>
void launch_brick(gf_ctx* c, const void* h, int force, Ctl* ctl, void* dst, int nact) {
    const Layout& L = c->L;
    const size_t lds = brick_lds(L.n[0], L.n[1], L.n[2], L.bk.by, L.bk.bz, sizeof(T));
#define GF_BRICK(NTB)                                                                                  \
    case NTB:                                                                                          \
        hipLaunchKernelGGL((k_update_measure_brick<T, NE, NTB>), dim3(loop_blocks(L), nact), dim3(NTB), lds, \
                           c->st, links_of<T, NE>(c), reinterpret_cast<const cx<T>*>(h), cxp<T>(dst), L.ps,   \
                           c->geom, L.bk, c->part, ctl, bt(c), force);                                  \
        break;
    switch (L.bk_threads) {
        GF_BRICK(256)
        GF_BRICK(512)
        GF_BRICK(768)
        GF_BRICK(1024)
        default:
            break;
    }
#undef GF_BRICK
}

template <typename T, int NE>
void launch_loop_kernel(gf_ctx* c, const void* h, int force, Ctl* ctl, void* dst, int nact) {
    const Layout& L = c->L;
    if (L.zb == -1) {
        launch_brick<T, NE>(c, h, force, ctl, dst, nact);
        return;
    }
    // 32-bit load offsets while the links' array spans less than 4 GiB (the transform's array is smaller)
    const bool o32 = (size_t)4 * NE * L.ps * sizeof(cx<T>) < ((size_t)1 << 32);
    auto kern = L.zb == 0 ? (o32 ? k_update_measure<T, NE, true, true> : k_update_measure<T, NE, true, false>)
                          : (o32 ? k_update_measure<T, NE, false, true> : k_update_measure<T, NE, false, false>);
    hipLaunchKernelGGL(kern, dim3(loop_blocks(L), nact), dim3(kFusedThreads), 0, c->st, links_of<T, NE>(c),
                       reinterpret_cast<const cx<T>*>(h), cxp<T>(dst), L.ps, c->geom, c->part, ctl, bt(c), L.zb,
                       force);
}

// Standalone measurement of the current links (transform in buffer k & 1): Delta -> D, theta and F.
template <typename T, int NE>
void launch_measure_t(gf_ctx* c) {
    tstart(c, GF_K_DIVERGENCE);
    launch_loop_kernel<T, NE>(c, c->Hb[cur(c)], 1, c->ctl, c->D, 1);
    tstop(c);
    tstart(c, GF_K_FINALIZE);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, c->st, c->part, c->L.nblk_fused, inv3v(c), inv12v(c),
                       c->ctl, 0, Batch{nullptr, 0});
    tstop(c);
}

// Update of the current links from (alpha/2) Delta~ packed in Q: H <- reunitarize(g H) in place.
template <typename T, int NE>
void launch_update_t(gf_ctx* c) {
    const Layout& L = c->L;
    tstart(c, GF_K_UPDATE);
    hipLaunchKernelGGL(k_h_update<T>, dim3(L.nblk), dim3(kSiteThreads), 0, c->st, reinterpret_cast<const cx<T>*>(c->Q),
                       L.ps, cxp<T>(c->Hb[cur(c)]), L.vol, exact_exp(c));
    tstop(c);
}

// Loop kernel after update k (transform of k + 1 updates): divergence -> D, partials.
template <typename T, int NE>
void launch_fused_t(gf_ctx* c, long long k) {
    tstart(c, GF_K_UPDATE_MEASURE);
    launch_loop_kernel<T, NE>(c, c->Hb[(k + 1) & 1], 0, c->ctl, c->D, c->nact);
    tstop(c);
}

template <typename T, int NE>
void launch_pack_t(gf_ctx* c, const double* src) {
    hipLaunchKernelGGL((k_pack<T, NE>), dim3(c->L.nblk), dim3(kSiteThreads), 0, c->st, src, links_of<T, NE>(c),
                       c->L.vol, sizeof(T) == 4 ? 1 : 0);
}
template <typename T, int NE>
void launch_unpack_t(gf_ctx* c, double* dst) {
    hipLaunchKernelGGL((k_unpack_h<T, NE>), dim3(c->L.nblk_fused), dim3(kSiteThreads), 0, c->st,
                       links_of<T, NE>(c), reinterpret_cast<const cx<T>*>(c->Hb[cur(c)]), c->geom, dst);
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
    const double coef = 0.5 * c->p.alpha * 16.0 / (double)c->L.vol;
    if (c->L.fp32) {
        launch_xy<float, false>(c, c->D, c->Q, 0, true);
        if (c->net_this)
            hipLaunchKernelGGL(k_mlp_table<float>, dim3((c->L.ntuples + kTableTuplesPerBlock - 1) / kTableTuplesPerBlock), dim3(256), 0, c->st, c->mlp,
                               reinterpret_cast<const float*>(c->sin2), c->tg, coef, c->ctl, 0,
                               reinterpret_cast<float*>(c->mtab));
        launch_zt<float>(c, c->Q, 0);
        launch_gauge_pass<float>(c, 0, c->Hb[k & 1], c->Hb[(k + 1) & 1]);
    } else {
        launch_xy<double, false>(c, c->D, c->Q, 0, true);
        if (c->net_this)
            hipLaunchKernelGGL(k_mlp_table<double>, dim3((c->L.ntuples + kTableTuplesPerBlock - 1) / kTableTuplesPerBlock), dim3(256), 0, c->st, c->mlp,
                               reinterpret_cast<const double*>(c->sin2), c->tg, coef, c->ctl, 0,
                               reinterpret_cast<double*>(c->mtab));
        launch_zt<double>(c, c->Q, 0);
        launch_gauge_pass<double>(c, 0, c->Hb[k & 1], c->Hb[(k + 1) & 1]);
    }
    GF_DISPATCH(c, launch_fused_t, c, k);
    return launched(c, "loop launch");
}

gf_status loop_finalize(gf_ctx* c) {
    tstart(c, GF_K_FINALIZE);
    hipLaunchKernelGGL(k_finalize, dim3(1, c->nact), dim3(256), 0, c->st, c->part, c->L.nblk_fused, inv3v(c),
                       inv12v(c), c->ctl, 1, bt(c));
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
template <typename T, int NE>
void raise_lds_brick() {
    const void* fns[] = {
        reinterpret_cast<const void*>(&k_update_measure_brick<T, NE, 256>),
        reinterpret_cast<const void*>(&k_update_measure_brick<T, NE, 512>),
        reinterpret_cast<const void*>(&k_update_measure_brick<T, NE, 768>),
        reinterpret_cast<const void*>(&k_update_measure_brick<T, NE, 1024>),
    };
    for (const void* f : fns) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsMax);
}

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
    raise_lds_brick<double, 9>();
    raise_lds_brick<double, 6>();
    raise_lds_brick<float, 9>();
    raise_lds_brick<float, 6>();
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
void gauge_unpack(gf_ctx* c, const void* rows, void* dst) {
    hipLaunchKernelGGL(k_gauge_unpack<T>, dim3(c->L.nblk), dim3(kSiteThreads), 0, c->st,
                       reinterpret_cast<const cx<T>*>(rows), reinterpret_cast<double*>(dst), c->L.vol);
}

// Forward FFT of Q, filter, and either the plain inverse (x, y) pass (gauge null) or the gauge pass writing
// g itself (rows 1-2) to gauge.
template <typename T>
void stage_spectral(gf_ctx* c, void* gauge) {
    launch_xy<T, false>(c, c->Q, c->Q, 1, false);
    launch_zt<T>(c, c->Q, 1);
    if (gauge)
        launch_gauge_pass<T>(c, 1, nullptr, gauge);
    else
        launch_xy<T, true>(c, c->Q, c->Q, 1, false);
}

// ------------------------------------------------------------- autotuning
// The compile-time FFT kernels come in several tilings per plane shape ((x, y):
// planes per block; (z, t): x columns per block). On the first context of a
// shape and precision in a process, each alternative is timed on the
// context's own buffers (two launches to warm up, then ten) and the fastest
// is kept for every later context of that shape and precision. The tilings
// compute bitwise the same transform.
struct TuneKey {
    int n[4];
    bool fp32;
    bool operator<(const TuneKey& o) const {
        for (int i = 0; i < 4; ++i)
            if (n[i] != o.n[i]) return n[i] < o.n[i];
        return fp32 < o.fp32;
    }
};
struct Tuned {
    int G, bx, zb;  // (x, y) planes per block, (z, t) columns per block, loop-kernel z grouping
};
std::map<TuneKey, Tuned> g_tuned;
std::mutex g_tuned_mu;

std::vector<int> xy_candidates(const Layout& L) {
    std::vector<int> v;
    const int nzt = L.n[2] * L.n[3];
#define GF_X(A, B, GG) \
    if (L.n[0] == A && L.n[1] == B && GG <= nzt && nzt % GG == 0) v.push_back(GG);
    GF_XY_CASES(GF_X)
#undef GF_X
    return v;
}

std::vector<int> zt_candidates(const Layout& L) {
    std::vector<int> v;
    if (const int rb = zt_reg_bx(L)) return {rb};  // one kernel, no tiling to choose
#define GF_X(A, B, BB) \
    if (L.n[2] == A && L.n[3] == B && L.n[0] % BB == 0) v.push_back(BB);
    if (L.fp32) {
        GF_ZT_CASES_F32(GF_X)
    } else {
        GF_ZT_CASES_F64(GF_X)
    }
#undef GF_X
    return v;
}

constexpr int kTuneReps = 10;
constexpr int kTuneRounds = 3;

template <typename T>
double time_pass(gf_ctx* c, bool xy) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreateWithFlags(&a, hipEventDisableSystemFence) != hipSuccess ||
        hipEventCreateWithFlags(&b, hipEventDisableSystemFence) != hipSuccess)
        return 1e30;
    auto run = [&]() {
        if (xy)
            launch_xy<T, false>(c, c->D, c->Q, 1, false);
        else
            launch_zt<T>(c, c->Q, 1);
    };
    run();
    run();
    (void)hipEventRecord(a, c->st);
    for (int i = 0; i < kTuneReps; ++i) run();
    (void)hipEventRecord(b, c->st);
    float ms = 1e30f;
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(&ms, a, b) != hipSuccess)
        ms = 1e30f;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms;
}

// Traversals the loop kernel can take on this shape: z groupings (1 always), 0 (blocks step through t)
// when the (x, y, z) volume is a multiple of 64 sites, t has at least 4 steps and there are at least 32
// blocks, and -1 (bricks) where the shape has a brick geometry.
std::vector<int> zb_candidates(const Layout& L) {
    std::vector<int> v{1};
    if (L.bk_threads > 0) v.push_back(-1);
    const int64_t vs = (int64_t)L.n[0] * L.n[1] * L.n[2];
    if (vs % kFusedSites == 0 && L.n[3] >= 4 && vs / kFusedSites >= 32) v.push_back(0);
    if ((L.n[0] * L.n[1]) % kFusedSites != 0) return v;
    for (int z : {2, 4, 8})
        if (L.n[2] % z == 0 && L.n[2] > z) v.push_back(z);
    return v;
}

template <typename T, int NE>
void time_loop_t(gf_ctx* c, double& ms_out) {
    // trial launches on the current links: divergence -> Q, partials of a scratch control-block head
    auto run = [&]() { launch_loop_kernel<T, NE>(c, c->Hb[cur(c)], 1, c->tune_ctl, c->Q, 1); };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ms_out = 1e30;
    if (hipEventCreateWithFlags(&e0, hipEventDisableSystemFence) != hipSuccess ||
        hipEventCreateWithFlags(&e1, hipEventDisableSystemFence) != hipSuccess)
        return;
    run();
    run();
    (void)hipEventRecord(e0, c->st);
    for (int i = 0; i < kTuneReps; ++i) run();
    (void)hipEventRecord(e1, c->st);
    float ms = 1e30f;
    if (hipGetLastError() == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
        hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
        ms_out = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

gf_status autotune(gf_ctx* c) {
    if (generic_fft(c) || c->cs != 0) return GF_OK;
    TuneKey key{};
    for (int i = 0; i < 4; ++i) key.n[i] = c->L.n[i];
    key.fp32 = c->L.fp32;
    {
        std::lock_guard<std::mutex> lock(g_tuned_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            set_xy_tile(c->L, it->second.G);
            set_zt_tile(c->L, it->second.bx);
            c->L.zb = it->second.zb;
            return GF_OK;
        }
    }
    int bestG = c->L.G, bestB = c->L.bx;
    const std::vector<int> xs = xy_candidates(c->L), zs = zt_candidates(c->L);
    // Each alternative is timed in kTuneRounds rounds, the order reversed every round so that no place
    // in the order is favoured (clocks still ramping up, caches still cold), and judged by its best round.
    auto pick = [&](const std::vector<int>& cand, bool xy, int& bestv) {
        std::vector<double> t(cand.size(), 1e30);
        for (int r = 0; r < kTuneRounds; ++r)
            for (size_t j = 0; j < cand.size(); ++j) {
                const size_t i = r % 2 == 0 ? j : cand.size() - 1 - j;
                if (xy)
                    set_xy_tile(c->L, cand[i]);
                else
                    set_zt_tile(c->L, cand[i]);
                t[i] = std::min(t[i], c->L.fp32 ? time_pass<float>(c, xy) : time_pass<double>(c, xy));
            }
        bestv = cand[std::min_element(t.begin(), t.end()) - t.begin()];
    };
    if (xs.size() > 1) pick(xs, true, bestG);
    set_xy_tile(c->L, bestG);
    if (zs.size() > 1) pick(zs, false, bestB);
    set_zt_tile(c->L, bestB);
    int bestZ = 1;
    const std::vector<int> zbs = zb_candidates(c->L);
    if (zbs.size() > 1) {
        // trial launches write Q, the block partials and a scratch control-block head; D, the control
        // block, the links and the transform are left as they are
        (void)hipMemsetAsync(c->tune_ctl, 0, offsetof(Ctl, hist_theta), c->st);
        std::vector<double> tz(zbs.size(), 1e30);
        for (int r = 0; r < kTuneRounds; ++r)
            for (size_t j = 0; j < zbs.size(); ++j) {
                const size_t i = r % 2 == 0 ? j : zbs.size() - 1 - j;
                c->L.zb = zbs[i];
                double t = 1e30;
                GF_DISPATCH(c, time_loop_t, c, t);
                tz[i] = std::min(tz[i], t);
            }
        bestZ = zbs[std::min_element(tz.begin(), tz.end()) - tz.begin()];
    }
    c->L.zb = bestZ;
    (void)hipGetLastError();
    std::lock_guard<std::mutex> lock(g_tuned_mu);
    g_tuned[key] = {bestG, bestB, bestZ};
    return check_hip(c, hipStreamSynchronize(c->st), "autotune sync");
}

// After its r-th rejected step the network pauses for 2^r plain updates; after
// kMaxRejects rejections it stays off.
constexpr int kMaxRejects = 6;

gf_status set_guard(gf_ctx* c, int on) {
    hipLaunchKernelGGL(k_set_guard, dim3(1), dim3(64), 0, c->st, c->ctl, on);
    return launched(c, "set_guard launch");
}

// Up to n learned updates under the device guard: the reduction that follows
// an update stops the loop if theta grew, F dropped or theta is not finite.
// A stopped update is undone (the links before it are still in the other
// link buffer), theta and F are measured again and a plain Fourier-
// accelerated update is taken in its place.
gf_status learned_chunk(gf_ctx* c, int64_t n) {
    gf_status s = set_guard(c, 1);
    c->net_this = true;
    for (int64_t i = 0; i < n && s == GF_OK; ++i) s = one_iteration(c, c->k_host + i);
    c->net_this = false;
    if (s == GF_OK) s = loop_finalize(c);
    if (s == GF_OK) s = read_head(c);
    if (s != GF_OK) return s;
    if (!c->h_head->rejected) return GF_OK;
    ++c->fallbacks;
    if (++c->rejects >= kMaxRejects) c->net_on = false;
    c->net_pause = 1ll << c->rejects;
    const long long k0 = c->h_head->iters - 1;
    hipLaunchKernelGGL(k_rollback, dim3(1), dim3(64), 0, c->st, c->ctl, k0);
    c->k_host = k0;
    s = launched(c, "rollback launch");
    if (s == GF_OK) s = set_guard(c, 0);
    if (s == GF_OK) s = launch_measure(c);
    if (s == GF_OK) s = read_head(c);
    if (s == GF_OK && !c->h_head->done) s = one_iteration(c, k0);
    if (s == GF_OK) s = loop_finalize(c);
    if (s == GF_OK) s = read_head(c);
    return s;
}

gf_status run_loop(gf_ctx* c, double tol, int64_t max_iter, gf_result* r, bool unpack = true) {
    const auto t0 = std::chrono::steady_clock::now();
    gf_status s = set_tol(c, tol);
    if (s == GF_OK) s = read_head(c);
    if (s != GF_OK) return s;
    const long long start = c->h_head->iters;
    while (!c->h_head->done && c->h_head->iters - start < max_iter) {
        const int64_t left = max_iter - (c->h_head->iters - start);
        int64_t k = std::min<int64_t>(left, c->p.check_every);
        if (c->net_on && c->net_pause == 0) {
            s = learned_chunk(c, k);
            if (s != GF_OK) return s;
            continue;
        }
        if (c->net_on) {  // paused after a rejection: plain updates, counted down
            k = std::min<int64_t>(k, c->net_pause);
            c->net_pause -= k;
        }
        for (int64_t i = 0; i < k && s == GF_OK; ++i) s = one_iteration(c, c->k_host + i);
        if (s == GF_OK) s = loop_finalize(c);
        if (s == GF_OK) s = read_head(c);
        if (s != GF_OK) return s;
    }
    if (unpack) {
        s = unpack_links(c, c->links_user);
        if (s == GF_OK) s = check_hip(c, hipStreamSynchronize(c->st), "sync");
        if (s != GF_OK) return s;
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (r) {
        r->iters = c->h_head->iters;
        r->theta = c->h_head->theta;
        r->F = c->h_head->F;
        r->phase = c->L.fp32 ? 0 : 1;
        r->fallbacks = c->fallbacks;
        r->seconds = secs;
    }
    if (c->h_head->numeric) return fail(c, GF_ENUMERIC, "theta is not finite");
    return GF_OK;
}

// Carve a plain (single-precision-class) context out of ws and set it up:
// tables, control block, links packed from the canonical d_links, the
// accumulated transform set to 1, and (if measure) theta and F of the input.
// Point c's buffers into ws as L lays them out (no device work, no allocation).
void carve(gf_ctx* c, const gf_params& p, const Layout& L, double* d_links, unsigned char* ws, hipStream_t st) {
    c->p = p;
    c->L = L;
    c->st = st;
    c->links_user = d_links;
    c->ws = ws;
    c->ctl = reinterpret_cast<Ctl*>(ws + L.off_ctl);
    c->tune_ctl = reinterpret_cast<Ctl*>(ws + L.off_tune);
    c->part = reinterpret_cast<double2*>(ws + L.off_part);
    c->sin2 = ws + L.off_sin2;
    for (int d = 0; d < 4; ++d) c->tw[d] = ws + L.off_tw + (size_t)d * kMaxExtent * 16;
    c->D = ws + L.off_d;
    c->Q = ws + L.off_q;
    c->U0 = ws + L.off_links;
    for (int i = 0; i < 2; ++i) c->Hb[i] = ws + L.off_h[i];
    c->mlp = L.learned ? reinterpret_cast<float*>(ws + L.off_mlp) : nullptr;
    c->mtab = L.learned ? ws + L.off_mtab : nullptr;
    for (int i = 0; i < 4; ++i) c->spec[i] = L.record ? ws + L.off_spec[i] : nullptr;
    c->rec = L.record ? reinterpret_cast<double*>(ws + L.off_rec) : nullptr;
    for (int d = 0; d < 4; ++d) {
        c->tg.n[d] = L.n[d];
        c->tg.h[d] = L.n[d] / 2 + 1;
    }
    c->tg.count = L.ntuples;
    c->k_host = 0;
    c->phase = L.fp32 ? 0 : 1;
    for (int d = 0; d < 4; ++d) {
        c->geom.n[d] = L.n[d];
        c->plan[d] = make_plan(L.n[d]);
    }
    c->geom.vol = L.vol;
    c->geom.stride[0] = 1;
    for (int d = 1; d < 4; ++d) c->geom.stride[d] = c->geom.stride[d - 1] * L.n[d - 1];
}

// Host data uploaded at set-up: the tables and the initial control-block head. A batch group shares
// one copy among its configurations and keeps it until its stream has been synchronised.
struct HostInit {
    std::vector<unsigned char> tables;
    std::vector<unsigned char> head;
};

void build_host_init(gf_ctx* c, HostInit& h) {
    if (c->L.fp32)
        fill_tables<float>(c, h.tables);
    else
        fill_tables<double>(c, h.tables);
    h.head.assign(kHeadBytes, 0);
    const double no_tol = -1.0;
    std::memcpy(h.head.data() + offsetof(Ctl, tol), &no_tol, sizeof(double));
}

// Set a plain context up in ws: tables, control block, links packed from the canonical d_links, the
// accumulated transform set to 1, and (if measure) theta and F of the input. With shared (a batch
// group's configurations) the host data come from there, h_head is the given slot and nothing is
// read back or waited for: the caller synchronises the stream before `shared` goes away.
gf_status init_plain(gf_ctx* c, const gf_params& p, const Layout& L, double* d_links, unsigned char* ws,
                     hipStream_t st, bool measure, HostInit* shared = nullptr, Ctl* head_slot = nullptr) {
    carve(c, p, L, d_links, ws, st);
    if (head_slot) {
        c->h_head = head_slot;
        c->own_head = false;
    } else if (hipHostMalloc(reinterpret_cast<void**>(&c->h_head), kHeadBytes) != hipSuccess) {
        c->h_head = nullptr;
        return fail(c, GF_EDEVICE, "hipHostMalloc of the control readback buffer failed");
    }
    std::memset(c->h_head, 0, kHeadBytes);
    raise_lds_limits();
    HostInit own;
    HostInit& h = shared ? *shared : own;
    if (h.tables.empty()) build_host_init(c, h);
    gf_status s;
    if ((s = check_hip(c, hipMemcpyAsync(c->sin2, h.tables.data(), h.tables.size(), hipMemcpyHostToDevice, c->st),
                       "table upload")) != GF_OK)
        return s;
    if ((s = check_hip(c, hipMemcpyAsync(c->ctl, h.head.data(), kHeadBytes, hipMemcpyHostToDevice, c->st),
                       "control upload")) != GF_OK)
        return s;
    GF_DISPATCH(c, launch_pack_t, c, c->links_user);
    s = launched(c, "pack launch");
    if (s == GF_OK) {  // no update applied yet: H = 1 in buffer 0
        if (L.fp32)
            hipLaunchKernelGGL(k_gauge_identity<float>, dim3(L.nblk), dim3(kSiteThreads), 0, c->st,
                               cxp<float>(c->Hb[0]), L.vol);
        else
            hipLaunchKernelGGL(k_gauge_identity<double>, dim3(L.nblk), dim3(kSiteThreads), 0, c->st,
                               cxp<double>(c->Hb[0]), L.vol);
        s = launched(c, "identity launch");
    }
    if (s == GF_OK && measure) s = launch_measure(c);
    if (s == GF_OK) s = autotune(c);
    if (shared) return s;
    if (s == GF_OK) s = read_head(c);
    if (s == GF_OK) {
        // hipMemcpyAsync from pageable memory may return before the copy is done: keep `own` alive until here.
        s = check_hip(c, hipStreamSynchronize(c->st), "sync");
    }
    return s;
}

void free_batch(BatchState* b);

void free_ctx(gf_ctx* c) {
    if (!c) return;
    for (int i = 0; i < 2; ++i) free_ctx(c->child[i]);
    if (c->batch) free_batch(c->batch);
    if (c->h_head) {
        (void)hipStreamSynchronize(c->st);
        if (c->own_head) (void)hipHostFree(c->h_head);
    }
    for (auto& e : c->ev) (void)hipEventDestroy(e);
    delete c;
}

gf_ctx* active(gf_ctx* c) { return c->L.mixed ? c->child[c->phase] : c; }

// GF_MIXED: float iterations (accumulating G) until theta < max(switch_theta,
// tol) or the float descent stalls, then U64 = G U0 G(x+mu)^dag in double and
// double iterations. tol < 0 means "apply max_iter updates" (gf_iterate).
// The float descent has stalled (its rounding floor is above the switch point) when theta has gone
// kStallIters updates without a new minimum while below kStallTheta, or kStallItersAny at any theta.
// theta is not monotone under steepest descent (F is): on thermalised fields it climbs back by two or
// three decades for some hundred updates before falling again, so a shorter window, or the drop over
// one check interval, hands over to double precision long before float has done its share.
constexpr double kStallTheta = 1e-6;
constexpr long long kStallIters = 200;
constexpr long long kStallItersAny = 2000;

struct StallTracker {
    double best = INFINITY;
    long long since = 0;  // updates since the last new minimum
    // theta after n more updates; true once the descent has stalled
    bool step(double theta, long long n) {
        if (theta < best) {
            best = theta;
            since = 0;
        } else {
            since += n;
        }
        return (theta < kStallTheta && since >= kStallIters) || since >= kStallItersAny;
    }
};

gf_status mixed_run(gf_ctx* c, double tol, int64_t max_iter, gf_result* r) {
    const auto t0 = std::chrono::steady_clock::now();
    gf_ctx* a = c->child[0];
    gf_ctx* b = c->child[1];
    int64_t left = max_iter;
    gf_status s = GF_OK;
    if (c->phase == 0) {
        const double sw = std::max(c->p.switch_theta, tol);
        StallTracker tracker;
        tracker.best = a->h_head->theta;
        bool stalled = false;
        while (left > 0 && !stalled) {
            const long long before = a->h_head->iters;
            s = run_loop(a, sw, std::min<int64_t>(left, a->p.check_every), nullptr, false);
            if (s != GF_OK) return fail(c, s, a->err);
            left -= a->h_head->iters - before;
            if (a->h_head->done) break;
            stalled = tracker.step(a->h_head->theta, a->h_head->iters - before);
        }
        if (a->h_head->numeric) return fail(c, GF_ENUMERIC, "theta is not finite");
        const bool reached = a->h_head->theta < sw;
        if ((tol > 0.0 && a->h_head->theta < tol) || (!reached && !stalled)) {
            // converged in float, or out of iterations before the hand-over
            s = unpack_links(a, c->links_user);
            if (s == GF_OK) s = check_hip(a, hipStreamSynchronize(a->st), "sync");
            if (s != GF_OK) return fail(c, s, a->err);
            if (r) {
                r->iters = a->h_head->iters;
                r->theta = a->h_head->theta;
                r->F = a->h_head->F;
                r->phase = 0;
                r->fallbacks = 0;
                r->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            }
            if (tol > 0.0 && !(a->h_head->theta < tol)) return fail(c, GF_ENOTCONV, "max_iter reached before theta < tol");
            return GF_OK;
        }
        // hand-over: the double child holds the input links; it takes over the float transform in double
        hipLaunchKernelGGL(k_promote_h, dim3(b->L.nblk), dim3(kSiteThreads), 0, b->st,
                           reinterpret_cast<const cx<float>*>(a->Hb[cur(a)]),
                           reinterpret_cast<cx<double>*>(b->Hb[cur(b)]), b->L.vol);
        s = launched(b, "hand-over launch");
        if (s == GF_OK) s = launch_measure(b);
        if (s == GF_OK) s = read_head(b);
        if (s != GF_OK) return fail(c, s, b->err);
        c->phase = 1;
    }
    s = run_loop(b, tol, left, nullptr, true);
    if (s != GF_OK) return fail(c, s, b->err);
    if (r) {
        r->iters = a->h_head->iters + b->h_head->iters;
        r->theta = b->h_head->theta;
        r->F = b->h_head->F;
        r->phase = 1;
        r->fallbacks = 0;
        r->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (tol > 0.0 && !b->h_head->done) return fail(c, GF_ENOTCONV, "max_iter reached before theta < tol");
    return GF_OK;
}


template <typename T, int NE>
void launch_plaquette_t(gf_ctx* c) {
    hipLaunchKernelGGL((k_plaquette_h<T, NE>), dim3(c->L.nblk), dim3(kSiteThreads), 0, c->st, links_of<T, NE>(c),
                       reinterpret_cast<const cx<T>*>(c->Hb[cur(c)]), c->geom, c->part);
    hipLaunchKernelGGL(k_plaquette_sum, dim3(1), dim3(256), 0, c->st, c->part, c->L.nblk,
                       1.0 / (18.0 * (double)c->L.vol), c->ctl);
}

// ------------------------------------------------------------- checkpoints
// A saved state is this header followed by a copy of the whole workspace
// (control block, history, tables, fields, both link buffers, accumulated
// gauge, network parameters), which holds no device addresses; it restores
// into any context made with the same parameters.
constexpr uint64_t kStateMagic = 0x3154415453464755ull;  // "UGFSTAT1"
constexpr size_t kStateHead = 256;

struct StateHeader {
    uint64_t magic;
    uint64_t total;
    int32_t dims[4];
    int32_t precision;
    uint32_t flags;
    int64_t k_host[3];  // this context, float child, double child
    int32_t phase, net_on, rejects, fallbacks;
    int64_t net_pause;
};
static_assert(sizeof(StateHeader) <= kStateHead, "state header too large");

StateHeader state_header(const gf_ctx* c) {
    StateHeader h{};
    h.magic = kStateMagic;
    h.total = c->L.total;
    std::copy(c->p.dims, c->p.dims + 4, h.dims);
    h.precision = c->p.precision;
    h.flags = c->p.flags;
    h.k_host[0] = c->k_host;
    for (int i = 0; i < 2; ++i) h.k_host[1 + i] = c->child[i] ? c->child[i]->k_host : 0;
    h.phase = c->phase;
    h.net_on = c->net_on ? 1 : 0;
    h.rejects = c->rejects;
    h.net_pause = c->net_pause;
    h.fallbacks = c->fallbacks;
    return h;
}

void restore_header(gf_ctx* c, const StateHeader& h) {
    c->k_host = h.k_host[0];
    for (int i = 0; i < 2; ++i)
        if (c->child[i]) c->child[i]->k_host = h.k_host[1 + i];
    c->phase = h.phase;
    c->net_on = h.net_on != 0;
    c->rejects = h.rejects;
    c->net_pause = h.net_pause;
    c->fallbacks = h.fallbacks;
}

// ----------------------------------------------------------------- batches
// Independent lattices of one shape form a group. A group's configurations
// share the compile-time FFT kernels and are advanced together: each loop
// kernel is one launch over the group's active configurations (blockIdx.y),
// each with its own slab of workspace, control block and stopping test.
// GF_MIXED groups run the float phase until every configuration has reached
// switch_theta (or stalled), hand each over to double precision, and polish.
struct BatchGroup {
    std::vector<int> idx;  // positions in the caller's arrays
    int nphase = 1;        // 2 for GF_MIXED
    gf_params q[2];
    Layout L[2];
    size_t cs[2] = {0, 0};   // bytes between consecutive configurations' slabs
    size_t off[2] = {0, 0};  // workspace offset of the first slab of each phase
    size_t off_act = 0, off_heads = 0;
    gf_ctx* drv[2] = {nullptr, nullptr};  // launches over the active configurations
    std::vector<gf_ctx*> view[2];         // one single-lattice context per configuration
    int* d_act = nullptr;
    unsigned char* d_heads = nullptr;
    int* h_act = nullptr;              // pinned
    unsigned char* h_heads = nullptr;  // pinned
    std::vector<unsigned char> h_views[2];  // the configurations' control-block heads (host)
    hipStream_t st = nullptr;          // the group's stream (shared when there are more groups than streams)
    hipEvent_t ev = nullptr;           // end of the group's last queued read-back
    // progress of gf_fix_until_batch
    enum Stage { kStart, kRun, kEnd, kDone } stage = kStart;
    int ph = 0;
    long long k = 0;   // updates every active configuration of the phase has applied
    int64_t left = 0;  // updates the group may still apply
    int64_t n_it = 0;  // updates in the chunk being read back
    bool waiting = false;
    std::vector<int> act;
    std::vector<long long> it0;
    std::vector<char> stalled;
    std::vector<StallTracker> tracker;  // float phase of GF_MIXED, as in the single-lattice path
};

struct BatchState {
    int n = 0;
    gf_params p{};
    size_t total = 0;
    std::vector<BatchGroup> g;
    // GF_FLAG_BATCH_FUSED: one launch per pass over every active configuration
    bool fused = false;
    size_t off_grp[2] = {0, 0}, off_seg = 0;  // workspace: shape tables per phase, segment table
    void* d_grp[2] = {nullptr, nullptr};
    int* d_seg = nullptr;  // first[4][n + 1], group[n], cfg[n]
    int* h_seg = nullptr;  // pinned staging of the segment table
    int thr[3] = {64, 64, 64};   // block sizes of the (x, y), (z, t) and gauge passes (largest shape)
    size_t lds[3] = {0, 0, 0};
    std::vector<hipStream_t> streams;  // the groups' streams, owned here
};

// Streams of a batch's shape groups: as many as the hardware queues a process gets besides the caller's
// stream (4 by default), so that the groups' streams are not multiplexed onto fewer queues than streams.
constexpr int kBatchStreams = 3;

void free_batch(BatchState* b) {
    if (b->h_seg) (void)hipHostFree(b->h_seg);
    for (auto& g : b->g) {
        for (int p = 0; p < 2; ++p) {
            for (gf_ctx* v : g.view[p]) free_ctx(v);
            free_ctx(g.drv[p]);
        }
        if (g.h_act) (void)hipHostFree(g.h_act);
        if (g.h_heads) (void)hipHostFree(g.h_heads);
        if (g.ev) (void)hipEventDestroy(g.ev);
    }
    for (hipStream_t st : b->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    delete b;
}

gf_status plan_batch(int32_t n, const gf_params* params, BatchState& b, std::string& err) {
    if (n < 1 || !params) {
        err = "a batch needs n >= 1 parameter sets";
        return GF_EINVAL;
    }
    const gf_params& p0 = params[0];
    for (int i = 0; i < n; ++i) {
        const gf_params& p = params[i];
        if (p.precision != p0.precision || p.alpha != p0.alpha || p.switch_theta != p0.switch_theta ||
            p.check_every != p0.check_every || p.flags != p0.flags) {
            err = "every configuration of a batch must share precision, alpha, switch_theta, check_every and flags";
            return GF_EINVAL;
        }
    }
    if (p0.flags & (GF_FLAG_LEARNED | GF_FLAG_RECORD_SPECTRA)) {
        err = "GF_FLAG_LEARNED and GF_FLAG_RECORD_SPECTRA are not available in a batch";
        return GF_EINVAL;
    }
    b.n = n;
    b.p = p0;
    b.g.clear();
    for (int i = 0; i < n; ++i) {
        BatchGroup* grp = nullptr;
        for (auto& g : b.g)
            if (std::equal(params[g.idx[0]].dims, params[g.idx[0]].dims + 4, params[i].dims)) grp = &g;
        if (!grp) {
            b.g.emplace_back();
            grp = &b.g.back();
        }
        grp->idx.push_back(i);
    }
    size_t o = 0;
    for (auto& g : b.g) {
        const gf_params& p = params[g.idx[0]];
        const int ng = (int)g.idx.size();
        g.nphase = p.precision == GF_MIXED ? 2 : 1;
        if (g.nphase == 2 && (!(p.switch_theta > 0.0) || !std::isfinite(p.switch_theta))) {
            err = "switch_theta must be positive and finite";
            return GF_EINVAL;
        }
        for (int ph = 0; ph < g.nphase; ++ph) {
            g.q[ph] = g.nphase == 2 ? mixed_child(p, ph) : p;
            gf_status s = plan_plain(&g.q[ph], g.L[ph], err);
            if (s != GF_OK) return s;
            g.cs[ph] = align_up(g.L[ph].total, kAlign);
            g.off[ph] = o;
            o += g.cs[ph] * ng;
        }
        g.off_act = o;
        o = align_up(o + (size_t)ng * sizeof(int), kAlign);
        g.off_heads = o;
        o = align_up(o + (size_t)ng * kHeadBytes, kAlign);
    }
    b.fused = (p0.flags & GF_FLAG_BATCH_FUSED) != 0;
    if (b.fused) {
        if ((int)b.g.size() > kMaxFusedGroups) {
            err = "GF_FLAG_BATCH_FUSED takes at most 8 lattice shapes";
            return GF_ENOTSUP;
        }
        for (auto& g : b.g)
            for (int ph = 0; ph < g.nphase; ++ph)
                if (g.L[ph].eptC != kEPT) {
                    err = "GF_FLAG_BATCH_FUSED: x-y planes too large for the fused inverse (x, y) pass";
                    return GF_ENOTSUP;
                }
        for (int ph = 0; ph < 2; ++ph) {
            b.off_grp[ph] = o;
            o = align_up(o + kMaxFusedGroups * sizeof(FusedGroup<double>), kAlign);
        }
        b.off_seg = o;
        o = align_up(o + (size_t)(4 * (n + 1) + 2 * n) * sizeof(int), kAlign);
    }
    b.total = o;
    return GF_OK;
}

// The per-shape tables of the fused passes (configuration 0 of each shape: the buffers carved for the
// group's launching context, drv).
template <typename T>
FusedGroup<T> fused_group(const BatchGroup& g, int ph) {
    const gf_ctx* d = g.drv[ph];
    const Layout& L = d->L;
    FusedGroup<T> f{};
    f.cs = g.cs[ph];
    f.ctl = d->ctl;
    f.part = d->part;
    f.U0 = reinterpret_cast<const cx<T>*>(d->U0);
    f.D = reinterpret_cast<cx<T>*>(d->D);
    f.Q = reinterpret_cast<cx<T>*>(d->Q);
    for (int i = 0; i < 2; ++i) f.H[i] = reinterpret_cast<cx<T>*>(d->Hb[i]);
    f.sin2 = reinterpret_cast<const T*>(d->sin2);
    for (int i = 0; i < 4; ++i) f.tw[i] = reinterpret_cast<const cx<T>*>(d->tw[i]);
    f.ps = L.ps;
    f.geom = d->geom;
    for (int i = 0; i < 4; ++i) f.plan[i] = d->plan[i];
    f.G = L.G;
    f.rs = L.rs;
    f.bx = L.bx;
    f.tsp = L.tsp;
    f.npart = L.nblk_fused;
    const bool no_fa = (d->p.flags & GF_FLAG_NO_FA) != 0;
    f.coef = 0.5 * d->p.alpha * (no_fa ? 1.0 : 16.0) / (double)L.vol;
    f.inv3v = 1.0 / (3.0 * (double)L.vol);
    f.inv12v = 1.0 / (12.0 * (double)L.vol);
    f.blocks[0] = 4 * L.n[2] * L.n[3] / L.G;
    f.blocks[1] = 4 * L.n[1] * (L.n[0] / L.bx);
    f.blocks[2] = L.n[2] * L.n[3];
    f.blocks[3] = L.nblk_fused;
    return f;
}

void raise_lds_fused() {
    static bool done = false;
    if (done) return;
    const int cap = (int)kLdsMax;
    const void* fns[] = {
        reinterpret_cast<const void*>(&k_fused_xy<double, kEPT>),
        reinterpret_cast<const void*>(&k_fused_zt<double, kEPT>),
        reinterpret_cast<const void*>(&k_fused_gauge<double, kEPT, 512>),
        reinterpret_cast<const void*>(&k_fused_gauge<double, kEPT, 1024>),
        reinterpret_cast<const void*>(&k_fused_xy<float, kEPT>),
        reinterpret_cast<const void*>(&k_fused_zt<float, kEPT>),
        reinterpret_cast<const void*>(&k_fused_gauge<float, kEPT, 512>),
        reinterpret_cast<const void*>(&k_fused_gauge<float, kEPT, 1024>),
    };
    for (const void* f : fns) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipGetLastError();
    done = true;
}

gf_status init_fused(gf_ctx* c, BatchState& b, unsigned char* ws) {
    raise_lds_fused();
    b.d_seg = reinterpret_cast<int*>(ws + b.off_seg);
    if (hipHostMalloc(reinterpret_cast<void**>(&b.h_seg), (size_t)(4 * (b.n + 1) + 2 * b.n) * sizeof(int)) !=
        hipSuccess) {
        b.h_seg = nullptr;
        return fail(c, GF_EDEVICE, "hipHostMalloc of the fused segment table failed");
    }
    for (auto& g : b.g)
        for (int ph = 0; ph < g.nphase; ++ph) {
            const Layout& L = g.drv[ph]->L;  // the tilings tuned for the shape
            b.thr[0] = std::max(b.thr[0], L.thrA);
            b.thr[1] = std::max(b.thr[1], L.thrB);
            b.thr[2] = std::max(b.thr[2], L.thrC);
            b.lds[0] = std::max(b.lds[0], L.ldsA);
            b.lds[1] = std::max(b.lds[1], L.ldsB);
            b.lds[2] = std::max(b.lds[2], L.ldsC);
        }
    const int nph = b.g.empty() ? 1 : b.g[0].nphase;
    for (int ph = 0; ph < nph; ++ph) {
        b.d_grp[ph] = ws + b.off_grp[ph];
        const bool fp32 = b.g[0].L[ph].fp32;
        std::vector<unsigned char> host(kMaxFusedGroups * sizeof(FusedGroup<double>), 0);
        for (size_t i = 0; i < b.g.size(); ++i) {
            if (fp32) {
                const FusedGroup<float> f = fused_group<float>(b.g[i], ph);
                std::memcpy(host.data() + i * sizeof(f), &f, sizeof(f));
            } else {
                const FusedGroup<double> f = fused_group<double>(b.g[i], ph);
                std::memcpy(host.data() + i * sizeof(f), &f, sizeof(f));
            }
        }
        GF_TRY_HIP(c, hipMemcpyAsync(b.d_grp[ph], host.data(), host.size(), hipMemcpyHostToDevice, c->st));
        GF_TRY_HIP(c, hipStreamSynchronize(c->st));  // host goes away
    }
    return GF_OK;
}

gf_status init_batch(gf_ctx* c, BatchState& b, double* const* d_links, unsigned char* ws, hipStream_t caller) {
    hipEvent_t ready = nullptr;  // the caller's links are written on its stream
    GF_TRY_HIP(c, hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    gf_status rs = check_hip(c, hipEventRecord(ready, caller), "event record");
    const int nst = std::min<int>(kBatchStreams, (int)b.g.size());
    for (int i = 0; i < nst && rs == GF_OK; ++i) {
        hipStream_t st = nullptr;
        rs = check_hip(c, hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "stream create");
        if (rs == GF_OK) b.streams.push_back(st);
        if (rs == GF_OK) rs = check_hip(c, hipStreamWaitEvent(st, ready, 0), "stream wait");
    }
    for (size_t i = 0; i < b.g.size() && rs == GF_OK; ++i) {
        BatchGroup& g = b.g[i];
        g.st = b.streams[i % b.streams.size()];
        rs = check_hip(c, hipEventCreateWithFlags(&g.ev, hipEventDisableTiming), "event create");
    }
    (void)hipEventDestroy(ready);
    if (rs != GF_OK) return rs;
    for (auto& g : b.g) {
        const hipStream_t st = g.st;
        const int ng = (int)g.idx.size();
        HostInit hinit[2];
        struct Drain {  // the uploads from hinit have finished before it goes away, on every return path
            hipStream_t st;
            ~Drain() { (void)hipStreamSynchronize(st); }
        } drain{st};
        for (int ph = 0; ph < g.nphase; ++ph) g.h_views[ph].assign((size_t)ng * kHeadBytes, 0);
        g.d_act = reinterpret_cast<int*>(ws + g.off_act);
        g.d_heads = ws + g.off_heads;
        if (hipHostMalloc(reinterpret_cast<void**>(&g.h_act), ng * sizeof(int)) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void**>(&g.h_heads), ng * kHeadBytes) != hipSuccess)
            return fail(c, GF_EDEVICE, "hipHostMalloc of the batch readback buffers failed");
        for (int ph = 0; ph < g.nphase; ++ph) {
            for (int i = 0; i < ng; ++i) {
                gf_ctx* v = new (std::nothrow) gf_ctx();
                if (!v) return fail(c, GF_EINVAL, "out of host memory");
                g.view[ph].push_back(v);
                // a GF_MIXED double slab keeps the input links in its buffer 0 until the hand-over
                const gf_status s =
                    init_plain(v, g.q[ph], g.L[ph], d_links[g.idx[i]], ws + g.off[ph] + i * g.cs[ph], st, ph == 0,
                               &hinit[ph], reinterpret_cast<Ctl*>(g.h_views[ph].data() + (size_t)i * kHeadBytes));
                if (s != GF_OK) return fail(c, s, v->err);
            }
            gf_ctx* d = new (std::nothrow) gf_ctx();
            if (!d) return fail(c, GF_EINVAL, "out of host memory");
            g.drv[ph] = d;
            carve(d, g.q[ph], g.L[ph], nullptr, ws + g.off[ph], st);
            set_xy_tile(d->L, g.view[ph][0]->L.G);  // the tiling tuned for this shape and precision
            set_zt_tile(d->L, g.view[ph][0]->L.bx);
            d->L.zb = g.view[ph][0]->L.zb;
            d->cs = g.cs[ph];
            d->act_dev = g.d_act;
        }
        GF_TRY_HIP(c, hipStreamSynchronize(st));  // reports a failed upload (drain repeats it harmlessly)
    }
    if (b.fused) return init_fused(c, b, ws);
    return GF_OK;
}

// Queue the read-back of every control block of phase ph (one gather kernel and one copy), and
// mark its end with the group's event.
gf_status enqueue_gather(gf_ctx* c, BatchGroup& g) {
    const int ng = (int)g.idx.size();
    hipLaunchKernelGGL(k_gather_heads, dim3(ng), dim3(64), 0, g.st,
                       reinterpret_cast<const unsigned char*>(g.view[g.ph][0]->ctl), g.cs[g.ph],
                       (int)(kHeadBytes / 8), reinterpret_cast<unsigned long long*>(g.d_heads));
    gf_status s = launched(c, "gather launch");
    if (s != GF_OK) return s;
    GF_TRY_HIP(c, hipMemcpyAsync(g.h_heads, g.d_heads, ng * kHeadBytes, hipMemcpyDeviceToHost, g.st));
    GF_TRY_HIP(c, hipEventRecord(g.ev, g.st));
    g.waiting = true;
    return GF_OK;
}

// Wait for the read-back and copy the control blocks into the views.
gf_status finish_gather(gf_ctx* c, BatchGroup& g) {
    GF_TRY_HIP(c, hipEventSynchronize(g.ev));
    g.waiting = false;
    const int ng = (int)g.idx.size();
    for (int i = 0; i < ng; ++i) {
        gf_ctx* v = g.view[g.ph][i];
        std::memcpy(v->h_head, g.h_heads + (size_t)i * kHeadBytes, kHeadBytes);
        v->k_host = v->h_head->iters;
    }
    return GF_OK;
}

struct BatchOutcome {
    gf_result r{};
    gf_status s = GF_OK;
    bool finished = false;
};

gf_status finish_config(gf_ctx* c, gf_ctx* v, int phase, long long iters_before, BatchOutcome& out, bool converged) {
    gf_status s = unpack_links(v, v->links_user);
    if (s != GF_OK) return fail(c, s, v->err);
    out.r.iters = iters_before + v->h_head->iters;
    out.r.theta = v->h_head->theta;
    out.r.F = v->h_head->F;
    out.r.phase = phase;
    out.r.fallbacks = 0;
    out.s = v->h_head->numeric ? GF_ENUMERIC : (converged ? GF_OK : GF_ENOTCONV);
    out.finished = true;
    return GF_OK;
}

double phase_tol(const gf_ctx* c, const BatchGroup& g, double tol) {
    return (g.nphase == 2 && g.ph == 0) ? std::max(c->p.switch_theta, tol) : tol;
}

// Queue the group's next piece of work on its stream (ending in a read-back when the host must look
// at the control blocks before going on).
gf_status advance_group(gf_ctx* c, BatchGroup& g, double tol, std::vector<BatchOutcome>& out) {
    const int ng = (int)g.idx.size();
    const bool mixed = g.nphase == 2;
    gf_status s = GF_OK;
    switch (g.stage) {
        case BatchGroup::kStart:  // arm the stopping test of the phase, then read every control block
            for (int i = 0; i < ng && s == GF_OK; ++i)
                if (!out[g.idx[i]].finished) s = set_tol(g.view[g.ph][i], phase_tol(c, g, tol));
            if (s == GF_OK) s = enqueue_gather(c, g);
            return s;
        case BatchGroup::kRun: {  // one chunk of updates over the active configurations
            gf_ctx* drv = g.drv[g.ph];
            std::copy(g.act.begin(), g.act.end(), g.h_act);
            GF_TRY_HIP(c, hipMemcpyAsync(g.d_act, g.h_act, g.act.size() * sizeof(int), hipMemcpyHostToDevice, g.st));
            drv->nact = (int)g.act.size();
            g.n_it = std::min<int64_t>(g.left, c->p.check_every);
            for (int64_t j = 0; j < g.n_it && s == GF_OK; ++j) s = one_iteration(drv, g.k + j);
            if (s == GF_OK) s = loop_finalize(drv);
            if (s == GF_OK) s = enqueue_gather(c, g);
            return s == GF_OK ? GF_OK : fail(c, s, drv->err);
        }
        case BatchGroup::kEnd: {  // hand-over to double precision, or the results of the phase
            const double tp = phase_tol(c, g, tol);
            for (int i = 0; i < ng; ++i) {
                BatchOutcome& o = out[g.idx[i]];
                if (o.finished) continue;
                gf_ctx* v = g.view[g.ph][i];
                const Ctl* h = v->h_head;
                if (mixed && g.ph == 0) {
                    g.it0[i] = h->iters;
                    const bool reached = h->theta < tp;
                    if (h->numeric || (tol > 0.0 && h->theta < tol) || (!reached && !g.stalled[i])) {
                        // converged in float, not finite, or out of iterations before the hand-over
                        s = finish_config(c, v, 0, 0, o, h->theta < tol);
                        if (s != GF_OK) return s;
                        continue;
                    }
                    gf_ctx* w = g.view[1][i];
                    hipLaunchKernelGGL(k_promote_h, dim3(w->L.nblk), dim3(kSiteThreads), 0, w->st,
                                       reinterpret_cast<const cx<float>*>(v->Hb[cur(v)]),
                                       reinterpret_cast<cx<double>*>(w->Hb[cur(w)]), w->L.vol);
                    s = launched(w, "hand-over launch");
                    if (s == GF_OK) s = launch_measure(w);
                    if (s != GF_OK) return fail(c, s, w->err);
                } else {
                    s = finish_config(c, v, mixed ? 1 : (v->L.fp32 ? 0 : 1), mixed ? g.it0[i] : 0, o, h->done != 0);
                    if (s != GF_OK) return s;
                }
            }
            if (mixed && g.ph == 0) {
                g.ph = 1;
                g.stage = BatchGroup::kStart;
            } else {
                g.stage = BatchGroup::kDone;
            }
            return GF_OK;
        }
        case BatchGroup::kDone:
            return GF_OK;
    }
    return GF_OK;
}

// Take in the read-back that advance_group queued.
gf_status absorb_group(gf_ctx* c, BatchGroup& g, std::vector<BatchOutcome>& out) {
    gf_status s = finish_gather(c, g);
    if (s != GF_OK) return s;
    const int ng = (int)g.idx.size();
    if (g.stage == BatchGroup::kStart) {
        g.act.clear();
        g.tracker.assign(ng, StallTracker{});
        for (int i = 0; i < ng; ++i) {
            const Ctl* h = g.view[g.ph][i]->h_head;
            g.tracker[i].best = h->theta;
            if (!out[g.idx[i]].finished && !h->done) g.act.push_back(i);
        }
        g.k = 0;  // every configuration of a phase starts from its own count 0
        g.stage = (g.act.empty() || g.left <= 0) ? BatchGroup::kEnd : BatchGroup::kRun;
        return GF_OK;
    }
    // a chunk of updates
    g.k += g.n_it;
    g.left -= g.n_it;
    std::vector<int> next;
    for (int i : g.act) {
        const Ctl* h = g.view[g.ph][i]->h_head;
        if (h->done || h->numeric) continue;
        if (h->iters != g.k) return fail(c, GF_EDEVICE, "batch configurations fell out of step");
        if (g.nphase == 2 && g.ph == 0) {
            g.stalled[i] = g.tracker[i].step(h->theta, g.n_it);
            if (g.stalled[i]) continue;
        }
        next.push_back(i);
    }
    g.act.swap(next);
    if (g.act.empty() || g.left <= 0) g.stage = BatchGroup::kEnd;
    return GF_OK;
}

// ---------------------------------------------------------------- fused batches
// Read every configuration's control block of phase ph into its view (one gather per shape, one wait).
gf_status fused_gather(gf_ctx* c, BatchState& b, int ph) {
    for (auto& g : b.g) {
        const int ng = (int)g.idx.size();
        hipLaunchKernelGGL(k_gather_heads, dim3(ng), dim3(64), 0, c->st,
                           reinterpret_cast<const unsigned char*>(g.view[ph][0]->ctl), g.cs[ph],
                           (int)(kHeadBytes / 8), reinterpret_cast<unsigned long long*>(g.d_heads));
        gf_status s = launched(c, "gather launch");
        if (s != GF_OK) return s;
        GF_TRY_HIP(c, hipMemcpyAsync(g.h_heads, g.d_heads, ng * kHeadBytes, hipMemcpyDeviceToHost, c->st));
    }
    GF_TRY_HIP(c, hipStreamSynchronize(c->st));
    for (auto& g : b.g)
        for (size_t i = 0; i < g.idx.size(); ++i) {
            gf_ctx* v = g.view[ph][i];
            std::memcpy(v->h_head, g.h_heads + i * kHeadBytes, kHeadBytes);
            v->k_host = v->h_head->iters;
        }
    return GF_OK;
}

// The segment table of the active configurations act = [(group, slot)] -> device (staged in pinned memory).
gf_status fused_table(gf_ctx* c, BatchState& b, int ph, const std::vector<std::pair<int, int>>& act, FusedTable& tb,
                      int total[4]) {
    const int n = (int)act.size();
    int* first[4];
    for (int p = 0; p < 4; ++p) first[p] = b.h_seg + p * (b.n + 1);
    int* grp = b.h_seg + 4 * (b.n + 1);
    int* cfg = grp + b.n;
    for (int p = 0; p < 4; ++p) first[p][0] = 0;
    for (int j = 0; j < n; ++j) {
        const BatchGroup& g = b.g[act[j].first];
        const Layout& L = g.drv[ph]->L;
        const int blocks[4] = {4 * L.n[2] * L.n[3] / L.G, 4 * L.n[1] * (L.n[0] / L.bx), L.n[2] * L.n[3],
                               L.nblk_fused};
        for (int p = 0; p < 4; ++p) first[p][j + 1] = first[p][j] + blocks[p];
        grp[j] = act[j].first;
        cfg[j] = act[j].second;
    }
    for (int p = 0; p < 4; ++p) total[p] = first[p][n];
    // the whole table in one copy (the previous chunk's kernels have finished: the host waited for them)
    GF_TRY_HIP(c, hipMemcpyAsync(b.d_seg, b.h_seg, (size_t)(4 * (b.n + 1) + 2 * b.n) * sizeof(int),
                                 hipMemcpyHostToDevice, c->st));
    for (int p = 0; p < 4; ++p) tb.first[p] = b.d_seg + p * (b.n + 1);
    tb.group = b.d_seg + 4 * (b.n + 1);
    tb.cfg = tb.group + b.n;
    tb.nseg = n;
    return GF_OK;
}

// One iteration k -> k + 1 of every active configuration: four launches.
template <typename T, int NE>
void fused_iteration_t(gf_ctx* c, BatchState& b, int ph, const FusedTable& tb, const int total[4], long long k) {
    const FusedGroup<T>* grp = reinterpret_cast<const FusedGroup<T>*>(b.d_grp[ph]);
    const int hp = (int)(k & 1);
    hipLaunchKernelGGL((k_fused_xy<T, kEPT>), dim3(total[0]), dim3(b.thr[0]), b.lds[0], c->st, grp, tb);
    hipLaunchKernelGGL((k_fused_zt<T, kEPT>), dim3(total[1]), dim3(b.thr[1]), b.lds[1], c->st, grp, tb,
                       (b.p.flags & GF_FLAG_NO_FA) ? 1 : 0);
    const int exact = (b.p.flags & GF_FLAG_EXACT_EXP) ? 1 : 0;
    if (b.thr[2] <= 512)
        hipLaunchKernelGGL((k_fused_gauge<T, kEPT, 512>), dim3(total[2]), dim3(b.thr[2]), b.lds[2], c->st, grp, tb,
                           hp, exact);
    else
        hipLaunchKernelGGL((k_fused_gauge<T, kEPT, 1024>), dim3(total[2]), dim3(b.thr[2]), b.lds[2], c->st, grp, tb,
                           hp, exact);
    hipLaunchKernelGGL((k_fused_loop<T, NE>), dim3(total[3]), dim3(kFusedThreads), 0, c->st, grp, tb, 1 - hp);
}

template <typename T>
void fused_finalize_t(gf_ctx* c, BatchState& b, int ph, const FusedTable& tb) {
    hipLaunchKernelGGL(k_fused_finalize<T>, dim3(tb.nseg), dim3(256), 0, c->st,
                       reinterpret_cast<const FusedGroup<T>*>(b.d_grp[ph]), tb);
}

// Every configuration to completion with one launch per pass: the phases of GF_MIXED advance in step
// (float until every configuration has reached switch_theta or stalled, then the hand-over, then double).
gf_status run_batch_fused(gf_ctx* c, BatchState& b, double tol, int64_t max_iter, std::vector<BatchOutcome>& out) {
    const int nph = b.g[0].nphase;
    const bool mixed = nph == 2;
    for (auto& g : b.g) {
        g.it0.assign(g.idx.size(), 0);
        g.stalled.assign(g.idx.size(), 0);
    }
    // everything below runs on the caller's stream, after the groups' set-up
    for (auto& g : b.g) {
        GF_TRY_HIP(c, hipEventRecord(g.ev, g.st));
        GF_TRY_HIP(c, hipStreamWaitEvent(c->st, g.ev, 0));
        for (int ph = 0; ph < nph; ++ph)
            for (gf_ctx* v : g.view[ph]) v->st = c->st;
    }
    int64_t left = max_iter;
    gf_status s = GF_OK;
    for (int ph = 0; ph < nph && s == GF_OK; ++ph) {
        const double tp = (mixed && ph == 0) ? std::max(c->p.switch_theta, tol) : tol;
        for (auto& g : b.g) {
            g.ph = ph;
            for (size_t i = 0; i < g.idx.size() && s == GF_OK; ++i)
                if (!out[g.idx[i]].finished) s = set_tol(g.view[ph][i], tp);
        }
        if (s == GF_OK) s = fused_gather(c, b, ph);
        if (s != GF_OK) return s;
        std::vector<std::pair<int, int>> act;
        for (size_t gi = 0; gi < b.g.size(); ++gi) {
            BatchGroup& g = b.g[gi];
            g.tracker.assign(g.idx.size(), StallTracker{});
            for (size_t i = 0; i < g.idx.size(); ++i) {
                const Ctl* h = g.view[ph][i]->h_head;
                g.tracker[i].best = h->theta;
                if (!out[g.idx[i]].finished && !h->done) act.emplace_back((int)gi, (int)i);
            }
        }
        long long k = 0;  // every configuration of a phase starts from its own count 0
        while (!act.empty() && left > 0 && s == GF_OK) {
            FusedTable tb{};
            int total[4];
            s = fused_table(c, b, ph, act, tb, total);
            if (s != GF_OK) return s;
            const int64_t n_it = std::min<int64_t>(left, c->p.check_every);
            for (int64_t j = 0; j < n_it; ++j) {
                if (b.g[0].L[ph].fp32) {
                    if (b.g[0].L[ph].ne == 6) fused_iteration_t<float, 6>(c, b, ph, tb, total, k + j);
                    else fused_iteration_t<float, 9>(c, b, ph, tb, total, k + j);
                } else {
                    if (b.g[0].L[ph].ne == 6) fused_iteration_t<double, 6>(c, b, ph, tb, total, k + j);
                    else fused_iteration_t<double, 9>(c, b, ph, tb, total, k + j);
                }
            }
            if (b.g[0].L[ph].fp32)
                fused_finalize_t<float>(c, b, ph, tb);
            else
                fused_finalize_t<double>(c, b, ph, tb);
            s = launched(c, "fused launch");
            if (s == GF_OK) s = fused_gather(c, b, ph);
            if (s != GF_OK) return s;
            k += n_it;
            left -= n_it;
            std::vector<std::pair<int, int>> next;
            for (const auto& a : act) {
                BatchGroup& g = b.g[a.first];
                const Ctl* h = g.view[ph][a.second]->h_head;
                if (h->done || h->numeric) continue;
                if (h->iters != k) return fail(c, GF_EDEVICE, "batch configurations fell out of step");
                if (mixed && ph == 0) {
                    g.stalled[a.second] = g.tracker[a.second].step(h->theta, n_it);
                    if (g.stalled[a.second]) continue;
                }
                next.push_back(a);
            }
            act.swap(next);
        }
        // end of the phase: hand-over to double precision, or the results
        for (auto& g : b.g) {
            for (size_t i = 0; i < g.idx.size() && s == GF_OK; ++i) {
                BatchOutcome& o = out[g.idx[i]];
                if (o.finished) continue;
                gf_ctx* v = g.view[ph][i];
                const Ctl* h = v->h_head;
                if (mixed && ph == 0) {
                    g.it0[i] = h->iters;
                    const bool reached = h->theta < tp;
                    if (h->numeric || (tol > 0.0 && h->theta < tol) || (!reached && !g.stalled[i])) {
                        s = finish_config(c, v, 0, 0, o, h->theta < tol);
                        continue;
                    }
                    gf_ctx* w = g.view[1][i];
                    hipLaunchKernelGGL(k_promote_h, dim3(w->L.nblk), dim3(kSiteThreads), 0, c->st,
                                       reinterpret_cast<const cx<float>*>(v->Hb[cur(v)]),
                                       reinterpret_cast<cx<double>*>(w->Hb[cur(w)]), w->L.vol);
                    s = launched(w, "hand-over launch");
                    if (s == GF_OK) s = launch_measure(w);
                    if (s != GF_OK) return fail(c, s, w->err);
                } else {
                    s = finish_config(c, v, mixed ? 1 : (v->L.fp32 ? 0 : 1), mixed ? g.it0[i] : 0, o, h->done != 0);
                }
            }
        }
    }
    return s;
}

// Every group to completion, side by side: queue each group's next piece of work on its stream,
// then take in the read-backs in turn.
gf_status run_batch(gf_ctx* c, BatchState& b, double tol, int64_t max_iter, std::vector<BatchOutcome>& out) {
    hipEvent_t ready = nullptr;  // the caller's stream is ordered before the groups' work
    GF_TRY_HIP(c, hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    gf_status s = check_hip(c, hipEventRecord(ready, c->st), "event record");
    for (auto& g : b.g) {
        const int ng = (int)g.idx.size();
        g.stage = BatchGroup::kStart;
        g.ph = 0;
        g.k = 0;
        g.left = max_iter;
        g.waiting = false;
        g.it0.assign(ng, 0);
        g.stalled.assign(ng, 0);
        if (s == GF_OK) s = check_hip(c, hipStreamWaitEvent(g.st, ready, 0), "stream wait");
    }
    (void)hipEventDestroy(ready);
    bool busy = true;
    while (s == GF_OK && busy) {
        busy = false;
        for (auto& g : b.g) {
            // phase ends queue work without a read-back: go on with the group until it waits or is done
            while (s == GF_OK && !g.waiting && g.stage != BatchGroup::kDone) s = advance_group(c, g, tol, out);
            busy = busy || g.stage != BatchGroup::kDone;
        }
        for (auto& g : b.g)
            if (s == GF_OK && g.waiting) s = absorb_group(c, g, out);
    }
    // the caller's stream waits for every group (the results are in the caller's link buffers)
    for (auto& g : b.g) {
        if (s != GF_OK) break;
        s = check_hip(c, hipEventRecord(g.ev, g.st), "event record");
        if (s == GF_OK) s = check_hip(c, hipStreamWaitEvent(c->st, g.ev, 0), "stream wait");
    }
    return s;
}
}  // namespace

// A plain streaming copy (16 bytes per lane, nontemporal): the bandwidth the device reaches on the
// simplest read-once / write-once traffic, against which the kernels' figures are read.
__global__ void __launch_bounds__(256) k_stream_copy(const cx<double>* __restrict__ a, cx<double>* __restrict__ b,
                                                     size_t n) {
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) nt_store(b + i, nt_load(a + i));
}

extern "C" {

size_t gf_workspace_bytes(const gf_params* params) {
    Layout L;
    std::string err;
    if (plan_layout(params, L, err) != GF_OK) return 0;
    return L.total;
}

// gf_init's work. heads: if set, two host slots of kHeadBytes for the control-block read-back (a plain
// context takes the first, a GF_MIXED context's children one each) instead of pinned host memory.
gf_status init_ctx(gf_ctx** out, const gf_params* params, void* d_links, void* d_workspace, size_t workspace_bytes,
                   void* stream, unsigned char* heads) {
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
        double* links = reinterpret_cast<double*>(d_links);
        unsigned char* ws = reinterpret_cast<unsigned char*>(d_workspace);
        hipStream_t st = reinterpret_cast<hipStream_t>(stream);
        auto slot = [&](int i) { return heads ? reinterpret_cast<Ctl*>(heads + (size_t)i * kHeadBytes) : nullptr; };
        if (!L.mixed) {
            s = init_plain(c, *params, L, links, ws, st, true, nullptr, slot(0));
        } else {
            c->p = *params;
            c->L = L;
            c->st = st;
            c->links_user = links;
            c->ws = ws;
            c->phase = 0;
            for (int i = 0; i < 2 && s == GF_OK; ++i) {
                c->child[i] = new (std::nothrow) gf_ctx();
                if (!c->child[i]) {
                    s = fail(c, GF_EINVAL, "out of host memory");
                    break;
                }
                const gf_params q = mixed_child(*params, i);
                Layout Lc;
                plan_plain(&q, Lc, err);
                // the double child keeps the input links untouched in its buffer 0 until the hand-over
                s = init_plain(c->child[i], q, Lc, links, ws + L.child_off[i], st, i == 0, nullptr, slot(i));
                if (s != GF_OK) c->err = c->child[i]->err;
            }
        }
        if (s != GF_OK) {
            g_init_error = c->err;
            free_ctx(c);
            return s;
        }
        *out = c;
        return GF_OK;
    } catch (...) {
        g_init_error = "unexpected host exception";
        return GF_EINVAL;
    }
}

gf_status gf_init(gf_ctx** out, const gf_params* params, void* d_links, void* d_workspace, size_t workspace_bytes,
                  void* stream) {
    return init_ctx(out, params, d_links, d_workspace, workspace_bytes, stream, nullptr);
}

// ----------------------------------------------------- entry point that allocates nothing
// The workspace of gf_fix_until_noalloc: a file-scope device array, one copy per GPU, held until the
// process ends. Host code takes its device address from hipGetSymbolAddress (once per device, with
// that device current) and never passes the array's own name to a kernel or a copy.
__device__ __align__(256) unsigned char scratch[GF_NOALLOC_SCRATCH_BYTES];

constexpr int kNoallocDevices = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ws[kNoallocDevices];
// control-block read-back slots (two: the children of a GF_MIXED context), per device
alignas(64) unsigned char g_noalloc_heads[kNoallocDevices][2 * kHeadBytes];

gf_status noalloc_workspace(void** ws, unsigned char** heads) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoallocDevices) {
        g_init_error = "gf_fix_until_noalloc: no current HIP device (or device index >= 64)";
        return GF_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ws[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            g_init_error = std::string("gf_fix_until_noalloc: hipGetSymbolAddress of the scratch failed: ") +
                           hipGetErrorString(e);
            return GF_EDEVICE;
        }
        g_noalloc_ws[dev] = p;
    }
    *ws = g_noalloc_ws[dev];
    *heads = g_noalloc_heads[dev];
    return GF_OK;
}

gf_status gf_fix_until_noalloc(const gf_params* params, void* d_links, void* stream, double theta_tol,
                               int64_t max_iter, gf_result* result) {
    try {
        Layout L;
        std::string err;
        gf_status s = plan_layout(params, L, err);
        if (s != GF_OK) {
            g_init_error = err;
            return s;
        }
        if (!d_links) {
            g_init_error = "links pointer is NULL";
            return GF_EINVAL;
        }
        if (L.total > (size_t)GF_NOALLOC_SCRATCH_BYTES) {
            g_init_error = "gf_fix_until_noalloc: this lattice and precision need " + std::to_string(L.total) +
                           " bytes of workspace; the scratch holds " + std::to_string((size_t)GF_NOALLOC_SCRATCH_BYTES) +
                           " (use gf_init with a workspace of your own)";
            return GF_ENOTSUP;
        }
        void* ws = nullptr;
        unsigned char* heads = nullptr;
        if ((s = noalloc_workspace(&ws, &heads)) != GF_OK) return s;
        gf_ctx* c = nullptr;
        s = init_ctx(&c, params, d_links, ws, GF_NOALLOC_SCRATCH_BYTES, stream, heads);
        if (s != GF_OK) return s;
        s = gf_fix_until(c, theta_tol, max_iter, result);
        if (s != GF_OK && s != GF_ENOTCONV) g_init_error = c->err;
        gf_destroy(c);
        return s;
    } catch (...) {
        g_init_error = "unexpected host exception";
        return GF_EINVAL;
    }
}

gf_status gf_iterate(gf_ctx* c, int64_t n, gf_result* r) {
    if (!c) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    if (n < 0) return fail(c, GF_EINVAL, "n must be >= 0");
    try {
        if (c->L.mixed) return mixed_run(c, -1.0, n, r);
        return run_loop(c, -1.0, n, r);
    } catch (...) {
        return fail(c, GF_EINVAL, "unexpected host exception");
    }
}

gf_status gf_advance(gf_ctx* c, int64_t n, gf_result* r) {
    if (!c) return GF_EINVAL;
    if (c->batch || c->L.mixed) return fail(c, GF_ESTATE, "gf_advance takes plain (non-mixed, non-batch) contexts");
    if (n < 0) return fail(c, GF_EINVAL, "n must be >= 0");
    try {
        return run_loop(c, -1.0, n, r, false);
    } catch (...) {
        return fail(c, GF_EINVAL, "unexpected host exception");
    }
}

gf_status gf_fix_until(gf_ctx* c, double tol, int64_t max_iter, gf_result* r) {
    if (!c) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    if (!(tol > 0.0)) return fail(c, GF_EINVAL, "theta_tol must be > 0");
    if (max_iter < 0) return fail(c, GF_EINVAL, "max_iter must be >= 0");
    try {
        if (c->L.mixed) return mixed_run(c, tol, max_iter, r);
        gf_status s = run_loop(c, tol, max_iter, r);
        if (s != GF_OK) return s;
        if (!c->h_head->done) return fail(c, GF_ENOTCONV, "max_iter reached before theta < tol");
        return GF_OK;
    } catch (...) {
        return fail(c, GF_EINVAL, "unexpected host exception");
    }
}

size_t gf_batch_workspace_bytes(int32_t n, const gf_params* params) {
    try {
        BatchState b;
        std::string err;
        return plan_batch(n, params, b, err) == GF_OK ? b.total : 0;
    } catch (...) {
        return 0;
    }
}

gf_status gf_init_batch(gf_ctx** out, int32_t n, const gf_params* params, double* const* d_links, void* d_workspace,
                        size_t workspace_bytes, void* stream) {
    try {
        if (!out) {
            g_init_error = "ctx output pointer is NULL";
            return GF_EINVAL;
        }
        *out = nullptr;
        BatchState* b = new (std::nothrow) BatchState();
        if (!b) {
            g_init_error = "out of host memory";
            return GF_EINVAL;
        }
        std::string err;
        gf_status s = plan_batch(n, params, *b, err);
        if (s == GF_OK) {
            // every lattice shape must plan on its own too (extents, plane sizes)
            for (int i = 0; i < n && s == GF_OK; ++i) {
                Layout L;
                s = plan_layout(&params[i], L, err);
            }
        }
        if (s == GF_OK && (!d_links || !d_workspace)) {
            err = "links or workspace pointer is NULL";
            s = GF_EINVAL;
        }
        for (int i = 0; s == GF_OK && i < n; ++i)
            if (!d_links[i]) {
                err = "links pointer " + std::to_string(i) + " is NULL";
                s = GF_EINVAL;
            }
        if (s == GF_OK && workspace_bytes < b->total) {
            err = "workspace too small: need " + std::to_string(b->total) + " bytes";
            s = GF_EINVAL;
        }
        if (s == GF_OK && (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) != 0) {
            err = "workspace must be 256-byte aligned";
            s = GF_EINVAL;
        }
        if (s != GF_OK) {
            g_init_error = err;
            delete b;
            return s;
        }
        gf_ctx* c = new (std::nothrow) gf_ctx();
        if (!c) {
            delete b;
            g_init_error = "out of host memory";
            return GF_EINVAL;
        }
        c->batch = b;
        c->p = b->p;
        c->st = reinterpret_cast<hipStream_t>(stream);
        s = init_batch(c, *b, d_links, reinterpret_cast<unsigned char*>(d_workspace), c->st);
        if (s != GF_OK) {
            g_init_error = c->err;
            free_ctx(c);
            return s;
        }
        *out = c;
        return GF_OK;
    } catch (...) {
        g_init_error = "unexpected host exception";
        return GF_EINVAL;
    }
}

gf_status gf_fix_until_batch(gf_ctx* c, double tol, int64_t max_iter, gf_result* results) {
    if (!c) return GF_EINVAL;
    if (!c->batch) return fail(c, GF_ESTATE, "not a batch context");
    if (!(tol > 0.0)) return fail(c, GF_EINVAL, "theta_tol must be > 0");
    if (max_iter < 0) return fail(c, GF_EINVAL, "max_iter must be >= 0");
    if (!results) return fail(c, GF_EINVAL, "results is NULL");
    try {
        const auto t0 = std::chrono::steady_clock::now();
        BatchState& b = *c->batch;
        std::vector<BatchOutcome> out(b.n);
        gf_status s = b.fused ? run_batch_fused(c, b, tol, max_iter, out) : run_batch(c, b, tol, max_iter, out);
        if (s != GF_OK) return s;
        s = check_hip(c, hipStreamSynchronize(c->st), "sync");
        if (s != GF_OK) return s;
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        gf_status worst = GF_OK;
        for (int i = 0; i < b.n; ++i) {
            results[i] = out[i].r;
            results[i].seconds = secs;
            if (out[i].s == GF_ENUMERIC) worst = GF_ENUMERIC;
            else if (out[i].s == GF_ENOTCONV && worst == GF_OK) worst = GF_ENOTCONV;
        }
        if (worst == GF_ENUMERIC) return fail(c, worst, "theta is not finite for at least one configuration");
        if (worst == GF_ENOTCONV) return fail(c, worst, "max_iter reached before theta < tol for at least one configuration");
        return GF_OK;
    } catch (...) {
        return fail(c, GF_EINVAL, "unexpected host exception");
    }
}

gf_status gf_quality(gf_ctx* c, double* theta, double* F) {
    if (!c) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    if (!theta || !F) return fail(c, GF_EINVAL, "null output");
    gf_ctx* a = active(c);
    gf_status s = read_head(a);
    if (s != GF_OK) return fail(c, s, a->err);
    *theta = a->h_head->theta;
    *F = a->h_head->F;
    return GF_OK;
}

gf_status gf_get_links(gf_ctx* c, void* d_out) {
    if (!c) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    if (!d_out) return fail(c, GF_EINVAL, "d_out is NULL");
    if (c->L.mixed) c = active(c);
    gf_status s = unpack_links(c, reinterpret_cast<double*>(d_out));
    if (s != GF_OK) return s;
    return check_hip(c, hipStreamSynchronize(c->st), "sync");
}

gf_status gf_plaquette(gf_ctx* c, double* plaquette) {
    if (!c) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    if (!plaquette) return fail(c, GF_EINVAL, "plaquette is NULL");
    gf_ctx* a = active(c);
    GF_DISPATCH(a, launch_plaquette_t, a);
    gf_status s = launched(a, "plaquette launch");
    if (s == GF_OK)
        s = check_hip(a, hipMemcpyAsync(plaquette, &a->ctl->plaquette, sizeof(double), hipMemcpyDeviceToHost, a->st),
                      "plaquette readback");
    if (s == GF_OK) s = check_hip(a, hipStreamSynchronize(a->st), "sync");
    return s == GF_OK ? GF_OK : fail(c, s, a->err);
}

gf_status gf_fft_tiling(gf_ctx* c, int32_t* xy_planes, int32_t* zt_columns) {
    if (!c || !xy_planes || !zt_columns) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    const gf_ctx* a = active(c);
    *xy_planes = a->L.G;
    *zt_columns = a->L.bx;
    return GF_OK;
}

gf_status gf_set_fft_tiling(gf_ctx* c, int32_t xy_planes, int32_t zt_columns) {
    if (!c) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    gf_ctx* a = active(c);
    if (generic_fft(a)) return fail(c, GF_ESTATE, "GF_FLAG_GENERIC_FFT keeps the runtime-shaped kernels' tiling");
    const std::vector<int> xs = xy_candidates(a->L), zs = zt_candidates(a->L);
    const bool okx = std::find(xs.begin(), xs.end(), (int)xy_planes) != xs.end();
    const bool okz = std::find(zs.begin(), zs.end(), (int)zt_columns) != zs.end();
    if (!okx || !okz) {
        std::string m = "compiled for this shape: xy_planes {";
        for (int v : xs) m += " " + std::to_string(v);
        m += " }, zt_columns {";
        for (int v : zs) m += " " + std::to_string(v);
        return fail(c, GF_EINVAL, m + " }");
    }
    set_xy_tile(a->L, xy_planes);
    set_zt_tile(a->L, zt_columns);
    return GF_OK;
}

gf_status gf_loop_traversal(gf_ctx* c, int32_t* z_group) {
    if (!c || !z_group) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    *z_group = active(c)->L.zb;
    return GF_OK;
}

gf_status gf_set_loop_traversal(gf_ctx* c, int32_t z_group) {
    if (!c) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    gf_ctx* a = active(c);
    const std::vector<int> v = zb_candidates(a->L);
    if (std::find(v.begin(), v.end(), (int)z_group) == v.end())
        return fail(c, GF_EINVAL,
                    "z_group must be 1, a divisor 2, 4, 8 of Nz below Nz (64 dividing Nx*Ny), 0 (t-march: 64 "
                    "dividing Nx*Ny*Nz, Nt >= 4, at least 32 blocks) or -1 (brick march, where the shape has "
                    "bricks)");
    a->L.zb = z_group;
    return GF_OK;
}

size_t gf_state_bytes(const gf_ctx* c) {
    if (!c || c->batch) return 0;
    return kStateHead + c->L.total;
}

gf_status gf_get_state(gf_ctx* c, void* d_out, size_t bytes) {
    if (!c) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    if (!d_out) return fail(c, GF_EINVAL, "d_out is NULL");
    if (bytes < gf_state_bytes(c)) return fail(c, GF_EINVAL, "state buffer too small");
    StateHeader h = state_header(c);
    unsigned char* o = reinterpret_cast<unsigned char*>(d_out);
    GF_TRY_HIP(c, hipMemcpyAsync(o, &h, sizeof(h), hipMemcpyHostToDevice, c->st));
    GF_TRY_HIP(c, hipMemcpyAsync(o + kStateHead, c->ws, c->L.total, hipMemcpyDeviceToDevice, c->st));
    return check_hip(c, hipStreamSynchronize(c->st), "sync");  // h must outlive the copy
}

gf_status gf_set_state(gf_ctx* c, const void* d_in, size_t bytes) {
    if (!c) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    if (!d_in) return fail(c, GF_EINVAL, "d_in is NULL");
    if (bytes < gf_state_bytes(c)) return fail(c, GF_EINVAL, "state buffer too small");
    const unsigned char* in = reinterpret_cast<const unsigned char*>(d_in);
    StateHeader h{};
    GF_TRY_HIP(c, hipMemcpyAsync(&h, in, sizeof(h), hipMemcpyDeviceToHost, c->st));
    GF_TRY_HIP(c, hipStreamSynchronize(c->st));
    const StateHeader mine = state_header(c);
    if (h.magic != kStateMagic || h.total != mine.total || h.precision != mine.precision || h.flags != mine.flags ||
        !std::equal(h.dims, h.dims + 4, mine.dims))
        return fail(c, GF_EINVAL, "state was not saved from a context with these parameters");
    GF_TRY_HIP(c, hipMemcpyAsync(c->ws, in + kStateHead, c->L.total, hipMemcpyDeviceToDevice, c->st));
    restore_header(c, h);
    gf_ctx* a = active(c);
    gf_status st = read_head(a);
    if (st == GF_OK) st = unpack_links(a, c->links_user);
    if (st == GF_OK) st = check_hip(a, hipStreamSynchronize(a->st), "sync");
    return st == GF_OK ? GF_OK : fail(c, st, a->err);
}

gf_status gf_history(gf_ctx* c, int64_t n, double* h_theta, double* h_F) {
    if (!c) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    if (!h_theta || !h_F) return fail(c, GF_EINVAL, "null output");
    if (c->L.mixed) c = active(c);
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
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    if (c->L.mixed) c = active(c);
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
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    if (c->L.mixed) c = active(c);
    if (!d_in || !d_out) return fail(c, GF_EINVAL, "null pointer");
    if (c->L.fp32) {
        field_pack<float>(c, d_in, c->Q);
        stage_spectral<float>(c, nullptr);
        field_unpack<float>(c, c->Q, d_out);
    } else {
        field_pack<double>(c, d_in, c->Q);
        stage_spectral<double>(c, nullptr);
        field_unpack<double>(c, c->Q, d_out);
    }
    gf_status s = launched(c, "filter launch");
    if (s != GF_OK) return s;
    return check_hip(c, hipStreamSynchronize(c->st), "sync");
}

gf_status gf_stage_gauge(gf_ctx* c, const void* d_in, void* d_out) {
    if (!c) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    if (c->L.mixed) c = active(c);
    if (!d_in || !d_out) return fail(c, GF_EINVAL, "null pointer");
    // g goes to the transform buffer the next update would overwrite anyway
    void* rows = c->Hb[1 - cur(c)];
    if (c->L.fp32) {
        field_pack<float>(c, d_in, c->Q);
        stage_spectral<float>(c, rows);
        gauge_unpack<float>(c, rows, d_out);
    } else {
        field_pack<double>(c, d_in, c->Q);
        stage_spectral<double>(c, rows);
        gauge_unpack<double>(c, rows, d_out);
    }
    gf_status s = launched(c, "gauge launch");
    if (s != GF_OK) return s;
    return check_hip(c, hipStreamSynchronize(c->st), "sync");
}

gf_status gf_stage_update(gf_ctx* c, const void* d_scaled) {
    if (!c) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    if (c->L.mixed) c = active(c);
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

gf_status gf_set_timing_mask(gf_ctx* c, uint32_t mask) {
    if (!c) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    if (c->L.mixed) {
        for (int i = 0; i < 2; ++i) {
            gf_status s = gf_set_timing_mask(c->child[i], mask);
            if (s != GF_OK) return s;
        }
        return GF_OK;
    }
    GF_TRY_HIP(c, hipStreamSynchronize(c->st));
    tdrain(c);
    c->timing = mask != 0;
    c->timing_mask = mask;
    for (int i = 0; i < GF_NKERNELS; ++i) {
        c->kt_ms[i] = 0.0;
        c->kt_n[i] = 0;
    }
    return GF_OK;
}

gf_status gf_set_timing(gf_ctx* c, int32_t enable) {
    return gf_set_timing_mask(c, enable ? (1u << GF_NKERNELS) - 1u : 0u);
}

gf_status gf_kernel_times(gf_ctx* c, int32_t n, double* h_ms_total, int64_t* h_counts) {
    if (!c) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    if (!h_ms_total || !h_counts || n < 0 || n > GF_NKERNELS) return fail(c, GF_EINVAL, "bad arguments");
    if (c->L.mixed) {
        double ms[GF_NKERNELS];
        int64_t cnt[GF_NKERNELS];
        for (int i = 0; i < n; ++i) {
            h_ms_total[i] = 0.0;
            h_counts[i] = 0;
        }
        for (int k = 0; k < 2; ++k) {
            gf_status s = gf_kernel_times(c->child[k], n, ms, cnt);
            if (s != GF_OK) return s;
            for (int i = 0; i < n; ++i) {
                h_ms_total[i] += ms[i];
                h_counts[i] += cnt[i];
            }
        }
        return GF_OK;
    }
    GF_TRY_HIP(c, hipStreamSynchronize(c->st));
    tdrain(c);
    for (int i = 0; i < n; ++i) {
        h_ms_total[i] = c->kt_ms[i];
        h_counts[i] = c->kt_n[i];
    }
    return GF_OK;
}

const char* gf_last_error(const gf_ctx* c) { return c ? c->err.c_str() : g_init_error.c_str(); }

gf_status gf_get_gauge(gf_ctx* c, void* d_out) {
    if (!c) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    if (!d_out) return fail(c, GF_EINVAL, "d_out is NULL");
    gf_ctx* a = active(c);
    if (a->L.fp32)
        gauge_unpack<float>(a, a->Hb[cur(a)], d_out);
    else
        gauge_unpack<double>(a, a->Hb[cur(a)], d_out);
    gf_status s = launched(a, "gauge unpack launch");
    if (s == GF_OK) s = check_hip(a, hipStreamSynchronize(a->st), "sync");
    return s == GF_OK ? s : fail(c, s, a->err);
}

gf_status gf_mlp_set_weights(gf_ctx* c, const float* d_params, int32_t enable) {
    if (!c) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    if (c->L.mixed || !c->mlp) return fail(c, GF_ESTATE, "context was created without GF_FLAG_LEARNED");
    if (enable && !d_params) return fail(c, GF_EINVAL, "d_params is NULL");
    if (d_params) GF_TRY_HIP(c, hipMemcpyAsync(c->mlp, d_params, kMlpParams * sizeof(float), hipMemcpyDeviceToDevice, c->st));
    GF_TRY_HIP(c, hipStreamSynchronize(c->st));
    c->net_on = enable != 0;
    c->rejects = 0;
    c->net_pause = 0;
    return GF_OK;
}

gf_status gf_mlp_multipliers(gf_ctx* c, void* d_out) {
    if (!c) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    if (c->L.mixed || !c->mlp) return fail(c, GF_ESTATE, "context was created without GF_FLAG_LEARNED");
    if (!d_out) return fail(c, GF_EINVAL, "d_out is NULL");
    const double coef = 0.5 * c->p.alpha * 16.0 / (double)c->L.vol;
    const dim3 grid((unsigned)((c->L.ntuples + kTableTuplesPerBlock - 1) / kTableTuplesPerBlock));
    if (c->L.fp32)
        hipLaunchKernelGGL(k_mlp_table<float>, grid, dim3(256), 0, c->st, c->mlp,
                           reinterpret_cast<const float*>(c->sin2), c->tg, coef, c->ctl, 1,
                           reinterpret_cast<float*>(d_out));
    else
        hipLaunchKernelGGL(k_mlp_table<double>, grid, dim3(256), 0, c->st, c->mlp,
                           reinterpret_cast<const double*>(c->sin2), c->tg, coef, c->ctl, 1,
                           reinterpret_cast<double*>(d_out));
    gf_status s = launched(c, "table launch");
    if (s == GF_OK) s = check_hip(c, hipStreamSynchronize(c->st), "sync");
    return s;
}

gf_status gf_record_spectra(gf_ctx* c, int64_t n, double probe_scale, double* d_records, double* h_theta) {
    if (!c) return GF_EINVAL;
    if (c->batch) return fail(c, GF_ESTATE, "a batch context only takes the batch calls");
    if (c->L.mixed || !c->rec) return fail(c, GF_ESTATE, "context was created without GF_FLAG_RECORD_SPECTRA");
    if (n < 1 || !d_records || !h_theta) return fail(c, GF_EINVAL, "bad arguments");
    if (!(probe_scale > 0.0) || !(probe_scale < 1.0)) return fail(c, GF_EINVAL, "probe_scale must be in (0, 1)");
    if (n + 1 > kHist) return fail(c, GF_EINVAL, "n too large");
    const bool was_on = c->net_on;
    c->net_on = false;
    gf_status s = set_tol(c, -1.0);
    if (s == GF_OK) s = set_guard(c, 0);
    if (s == GF_OK) s = read_head(c);
    const long long k0 = c->k_host;
    const size_t recn = (size_t)c->L.ntuples * 3;
    auto forward_passes = [&]() {  // spectrum of D into spec_capture (forward (x, y) and (z, t) passes into Q)
        if (c->L.fp32) {
            launch_xy<float, false>(c, c->D, c->Q, 1, true);
            launch_zt<float>(c, c->Q, 1);
        } else {
            launch_xy<double, false>(c, c->D, c->Q, 1, true);
            launch_zt<double>(c, c->Q, 1);
        }
        return launched(c, "spectrum launch");
    };
    for (int64_t i = 0; i <= n && s == GF_OK; ++i) {
        const long long k = k0 + i;
        c->spec_capture = c->spec[i & 1];
        if (i < n) {
            // probe: the update with every multiplier times probe_scale (captures the spectrum of step i) ...
            c->coef_scale = probe_scale;
            s = one_iteration(c, k);
            c->coef_scale = 1.0;
            c->spec_capture = c->spec[2 + (i & 1)];
            if (s == GF_OK) s = forward_passes();  // ... and the spectrum of its result
            c->spec_capture = nullptr;
            // undo it (the links of step i are still in the other buffer), re-measure, take the plain step
            if (s == GF_OK) {
                hipLaunchKernelGGL(k_rollback, dim3(1), dim3(64), 0, c->st, c->ctl, k);
                s = launched(c, "rollback launch");
            }
            c->k_host = k;
            if (s == GF_OK) s = launch_measure(c);
            if (s == GF_OK) s = one_iteration(c, k);
        } else {
            s = forward_passes();  // spectrum of the last iterate only
        }
        c->spec_capture = nullptr;
        if (s == GF_OK && i >= 1) {
            const int a = (i - 1) & 1, b = i & 1, pb = 2 + ((i - 1) & 1);
            if (c->L.fp32)
                hipLaunchKernelGGL(k_record_tuples<float>, dim3((c->L.ntuples + 255) / 256), dim3(256), 0, c->st,
                                   reinterpret_cast<const cx<float>*>(c->spec[a]),
                                   reinterpret_cast<const cx<float>*>(c->spec[b]),
                                   reinterpret_cast<const cx<float>*>(c->spec[pb]), c->L.ps, c->tg,
                                   d_records + (size_t)(i - 1) * recn);
            else
                hipLaunchKernelGGL(k_record_tuples<double>, dim3((c->L.ntuples + 255) / 256), dim3(256), 0, c->st,
                                   reinterpret_cast<const cx<double>*>(c->spec[a]),
                                   reinterpret_cast<const cx<double>*>(c->spec[b]),
                                   reinterpret_cast<const cx<double>*>(c->spec[pb]), c->L.ps, c->tg,
                                   d_records + (size_t)(i - 1) * recn);
            s = launched(c, "record launch");
        }
    }
    c->k_host = k0 + n;
    if (s == GF_OK) s = loop_finalize(c);
    if (s == GF_OK) s = read_head(c);
    if (s == GF_OK) s = unpack_links(c, c->links_user);
    c->net_on = was_on;
    if (s != GF_OK) return s;
    std::vector<double> th(kHist), f(kHist);
    GF_TRY_HIP(c, hipMemcpyAsync(th.data(), c->ctl->hist_theta, kHist * sizeof(double), hipMemcpyDeviceToHost, c->st));
    GF_TRY_HIP(c, hipStreamSynchronize(c->st));
    for (int64_t i = 0; i < n; ++i) h_theta[i] = th[(k0 + i) % kHist];
    return GF_OK;
}

// ----------------------------------------------------------- training
size_t gf_mlp_workspace_bytes(int64_t n_rows, int32_t n_samples) {
    if (n_rows < 1 || n_samples < 1) return 0;
    const size_t nb = (size_t)((n_rows + kBwdBlockRows - 1) / kBwdBlockRows);
    size_t o = 0;
    o = align_up(o + (size_t)n_rows * kMlpH * sizeof(float), kAlign);   // H1
    o = align_up(o + (size_t)n_rows * kMlpH * sizeof(float), kAlign);   // H2
    o = align_up(o + (size_t)n_rows * 2 * sizeof(float), kAlign);       // O
    o = align_up(o + (size_t)n_rows * 2 * sizeof(float), kAlign);       // dO
    o = align_up(o + nb * kMlpParams * sizeof(float), kAlign);          // block partial gradients
    o = align_up(o + (size_t)n_samples * sizeof(double), kAlign);       // sample losses
    return o;
}

namespace {
struct MlpWs {
    float *h1, *h2, *o, *dO, *gpart;
    double* sloss;
    int nb;
};
MlpWs carve_mlp(void* ws, int64_t n_rows, int32_t n_samples) {
    MlpWs w;
    unsigned char* b = reinterpret_cast<unsigned char*>(ws);
    w.nb = (int)((n_rows + kBwdBlockRows - 1) / kBwdBlockRows);
    size_t o = 0;
    w.h1 = reinterpret_cast<float*>(b + o);
    o = align_up(o + (size_t)n_rows * kMlpH * sizeof(float), kAlign);
    w.h2 = reinterpret_cast<float*>(b + o);
    o = align_up(o + (size_t)n_rows * kMlpH * sizeof(float), kAlign);
    w.o = reinterpret_cast<float*>(b + o);
    o = align_up(o + (size_t)n_rows * 2 * sizeof(float), kAlign);
    w.dO = reinterpret_cast<float*>(b + o);
    o = align_up(o + (size_t)n_rows * 2 * sizeof(float), kAlign);
    w.gpart = reinterpret_cast<float*>(b + o);
    o = align_up(o + (size_t)w.nb * kMlpParams * sizeof(float), kAlign);
    w.sloss = reinterpret_cast<double*>(b + o);
    (void)n_samples;
    return w;
}
void raise_mlp_lds() {
    static bool done = false;
    if (done) return;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mlp_backward), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)kBwdLds);
    done = true;
}
gf_status mlp_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return GF_OK;
    g_init_error = std::string(what) + ": " + hipGetErrorString(e);
    return GF_EDEVICE;
}
}  // namespace

gf_status gf_mlp_forward(const float* d_params, const float* d_x, int64_t n_rows, float* d_out, void* d_ws,
                         size_t ws_bytes, void* stream) {
    if (!d_params || !d_x || !d_out || !d_ws || n_rows < 1) return GF_EINVAL;
    if (ws_bytes < gf_mlp_workspace_bytes(n_rows, 1)) return GF_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    MlpWs w = carve_mlp(d_ws, n_rows, 1);
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((n_rows + 255) / 256)), dim3(256), 0, st, d_params, d_x, n_rows,
                       w.h1, w.h2, d_out);
    gf_status s = mlp_status(hipGetLastError(), "mlp forward");
    if (s == GF_OK) s = mlp_status(hipStreamSynchronize(st), "sync");
    return s;
}

gf_status gf_mlp_loss_grad(const float* d_params, const float* d_x, const float* d_tgt, const int32_t* d_offsets,
                           int32_t n_samples, int64_t n_rows, float* d_grad, void* d_ws, size_t ws_bytes,
                           void* stream, double* h_loss) {
    if (!d_params || !d_x || !d_tgt || !d_offsets || !d_grad || !d_ws || n_rows < 1 || n_samples < 1)
        return GF_EINVAL;
    if (ws_bytes < gf_mlp_workspace_bytes(n_rows, n_samples)) return GF_EINVAL;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    MlpWs w = carve_mlp(d_ws, n_rows, n_samples);
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((n_rows + 255) / 256)), dim3(256), 0, st, d_params, d_x, n_rows,
                       w.h1, w.h2, w.o);
    hipLaunchKernelGGL(k_mlp_loss, dim3(n_samples), dim3(256), 0, st, w.o, d_tgt, d_offsets, n_samples, w.dO, w.sloss);
    raise_mlp_lds();
    hipLaunchKernelGGL(k_mlp_backward, dim3(w.nb), dim3(256), kBwdLds, st, d_params, d_x, w.h1, w.h2, w.dO, n_rows,
                       w.gpart);
    hipLaunchKernelGGL(k_grad_reduce, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, w.gpart, w.nb, d_grad);
    gf_status s = mlp_status(hipGetLastError(), "mlp loss/gradient");
    if (s == GF_OK && h_loss) {
        std::vector<double> sl(n_samples);
        s = mlp_status(hipMemcpyAsync(sl.data(), w.sloss, n_samples * sizeof(double), hipMemcpyDeviceToHost, st),
                       "loss readback");
        if (s == GF_OK) s = mlp_status(hipStreamSynchronize(st), "sync");
        double t = 0.0;
        for (double v : sl) t += v;
        *h_loss = t / n_samples;
    }
    return s;
}

gf_status gf_mlp_adam(float* d_params, float* d_m, float* d_v, const float* d_grad, int64_t step, float lr,
                      void* stream) {
    if (!d_params || !d_m || !d_v || !d_grad || step < 1 || !(lr > 0.f)) return GF_EINVAL;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = (float)(1.0 - std::pow(0.9, (double)step)), c2 = (float)(1.0 - std::pow(0.999, (double)step));
    hipLaunchKernelGGL(k_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                       d_params, d_m, d_v, d_grad, lr, b1, b2, 1e-8f, c1, c2);
    return mlp_status(hipGetLastError(), "adam");
}

gf_status gf_mlp_train_step(float* d_params, float* d_m, float* d_v, int64_t step, float lr, const float* d_x,
                            const float* d_tgt, const int32_t* d_offsets, int32_t n_samples, int64_t n_rows,
                            float* d_grad, void* d_ws, size_t ws_bytes, void* stream, double* h_loss) {
    gf_status s = gf_mlp_loss_grad(d_params, d_x, d_tgt, d_offsets, n_samples, n_rows, d_grad, d_ws, ws_bytes, stream,
                                   h_loss);
    if (s != GF_OK) return s;
    return gf_mlp_adam(d_params, d_m, d_v, d_grad, step, lr, stream);
}

int32_t gf_mlp_param_count(void) { return kMlpParams; }

gf_status gf_mlp_make_samples(const double* d_records, int32_t n_records, const double* d_theta, int32_t first,
                              int32_t every, int32_t n_samples, int64_t k0, double probe_scale, const int32_t* dims,
                              float* d_x, float* d_tgt, void* stream) {
    if (!d_records || !d_theta || !dims || !d_x || !d_tgt || n_samples < 1 || every < 1 || first < 0 || k0 < 0)
        return GF_EINVAL;
    if (!(probe_scale > 0.0) || !(probe_scale < 1.0)) return GF_EINVAL;
    if ((int64_t)first + (int64_t)(n_samples - 1) * every > (int64_t)n_records - 2) return GF_EINVAL;
    TupleGeom tg;
    tg.count = 1;
    for (int d = 0; d < 4; ++d) {
        if (dims[d] < 2 || dims[d] % 2) return GF_EINVAL;
        tg.n[d] = dims[d];
        tg.h[d] = dims[d] / 2 + 1;
        tg.count *= tg.h[d];
    }
    const int64_t nrows = (int64_t)n_samples * tg.count;
    hipLaunchKernelGGL(k_make_samples, dim3((unsigned)((nrows + 255) / 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), d_records, d_theta, first, every, (long long)k0,
                       probe_scale, nrows, tg, d_x, d_tgt);
    return mlp_status(hipGetLastError(), "make samples");
}

void gf_destroy(gf_ctx* c) { free_ctx(c); }

gf_status gf_stream_copy(const void* d_src, void* d_dst, size_t bytes, void* stream) {
    if (!d_src || !d_dst || bytes % 16 || reinterpret_cast<uintptr_t>(d_src) % 16 ||
        reinterpret_cast<uintptr_t>(d_dst) % 16)
        return GF_EINVAL;
    const size_t n = bytes / 16;
    if (n == 0) return GF_OK;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       reinterpret_cast<hipStream_t>(stream), static_cast<const cx<double>*>(d_src),
                       static_cast<cx<double>*>(d_dst), n);
    return hipGetLastError() == hipSuccess ? GF_OK : GF_EDEVICE;
}

}  // extern "C"

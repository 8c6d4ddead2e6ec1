// libgf host side: the C ABI declared in include/gf.h.
//
// The context carves the caller's workspace into: a device control block
// (theta, F, stop flag, iteration count, history), per-block reduction
// partials, FFT twiddle and sin^2 tables, the four packed Delta fields and
// the structure-of-arrays links. Every kernel is queued on the caller's
// stream; the loop reads the control block back every check_every
// iterations, and kernels queued after the stop flag is set return at once,
// so the iterate is exactly the one the stopping rule selects.
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
#include "gf_kernels.hpp"

using namespace gf;

namespace {

constexpr int kEPT = 8;         // FFT elements held per thread per stage
constexpr int kMaxExtent = 64;  // largest supported extent
constexpr size_t kAlign = 256;

thread_local std::string g_init_error;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

bool is_2a3b(int n) {
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

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
    size_t ps;          // plane stride (elements)
    int nblk;           // site blocks
    bool fp32;
    int ne;             // 9 or 6
    // pass A
    int G, rs, thrA;
    size_t ldsA;
    // pass B
    int bx, tsp, thrB;
    size_t ldsB;
    // workspace offsets
    size_t off_ctl, off_part, off_sin2, off_tw, off_z, off_links, total;
};

int round64(int x) { return (x + 63) / 64 * 64; }

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
    if (vol > (int64_t)1 << 31) {
        err = "lattice too large";
        return GF_ENOTSUP;
    }
    if (p->precision < GF_FP64_18 || p->precision > GF_FP32_18) {
        err = p->precision == GF_MIXED ? "GF_MIXED is not available in this build" : "unknown precision";
        return p->precision == GF_MIXED ? GF_ENOTSUP : GF_EINVAL;
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
    L.ps = align_up((size_t)vol, 256);
    L.nblk = (int)((vol + kSiteThreads - 1) / kSiteThreads);
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2], nt = L.n[3];
    // Pass A: G planes per block, enough work per block, never straddling a field.
    const int nzt = nz * nt;
    L.G = 1;
    while (L.G * 2 <= nzt && nzt % (L.G * 2) == 0 && L.G * nx * ny < 512) L.G *= 2;
    L.rs = nx + 1;
    const int EA = L.G * nx * ny;
    L.thrA = std::min(1024, std::max(64, round64((EA + kEPT - 1) / kEPT)));
    L.ldsA = (size_t)(nx + ny) * csz + (size_t)L.G * ny * L.rs * csz;
    // Pass B: bx consecutive x columns, >= 64 contiguous bytes when possible.
    const size_t ldsCap = 80 * 1024;
    L.bx = 1;
    for (int b : {16, 8, 4, 2, 1}) {
        if (nx % b != 0) continue;
        const int E = b * nz * nt;
        const size_t lds = (size_t)(nz + nt) * csz + (size_t)nt * (nz * b + 1) * csz;
        if (E <= kEPT * 1024 && lds <= ldsCap && (size_t)b * csz <= 128) {
            L.bx = b;
            break;
        }
    }
    L.tsp = nz * L.bx + 1;
    const int EB = L.bx * nz * nt;
    if (EB > kEPT * 1024) {
        err = "z-t plane too large";
        return GF_ENOTSUP;
    }
    L.thrB = std::min(1024, std::max(64, round64((EB + kEPT - 1) / kEPT)));
    L.ldsB = (size_t)(nz + nt) * csz + (size_t)nt * L.tsp * csz;
    // Workspace.
    size_t o = 0;
    L.off_ctl = o;
    o = align_up(o + sizeof(Ctl), kAlign);
    L.off_part = o;
    o = align_up(o + (size_t)L.nblk * sizeof(double2), kAlign);
    L.off_sin2 = o;
    o = align_up(o + 4 * kMaxExtent * sizeof(double), kAlign);
    L.off_tw = o;
    o = align_up(o + 4 * kMaxExtent * 16, kAlign);
    L.off_z = o;
    o = align_up(o + 4 * L.ps * csz, kAlign);
    L.off_links = o;
    o = align_up(o + (size_t)4 * L.ne * L.ps * csz, kAlign);
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
    void* Z;
    void* links;
    FftPlan plan[4];
    Ctl* h_head;  // pinned host copy of the control block's leading scalars
    std::string err;
    // Optional per-kernel HIP-event timing (gf_set_timing / gf_kernel_times).
    bool timing = false;
    std::vector<hipEvent_t> ev;   // 2 per pending measurement
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

#define GF_TRY_HIP(c, call)                                       \
    do {                                                          \
        gf_status _s = check_hip((c), (call), #call);             \
        if (_s != GF_OK) return _s;                               \
    } while (0)

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

template <typename T, int NE>
Links<T, NE> links_of(gf_ctx* c) {
    return Links<T, NE>{reinterpret_cast<cx<T>*>(c->links), c->L.ps};
}

template <typename T>
gf_status launch_fft(gf_ctx* c, int force) {
    const Layout& L = c->L;
    cx<T>* Z = reinterpret_cast<cx<T>*>(c->Z);
    const cx<T>* tw[4];
    for (int i = 0; i < 4; ++i) tw[i] = reinterpret_cast<const cx<T>*>(c->tw[i]);
    const int nzt = L.n[2] * L.n[3];
    const int gridA = 4 * nzt / L.G;
    const int gridB = 4 * L.n[1] * (L.n[0] / L.bx);
    const double coef = 0.5 * c->p.alpha * ((c->p.flags & GF_FLAG_NO_FA) ? 1.0 : 16.0) / (double)L.vol;
    const int no_fa = (c->p.flags & GF_FLAG_NO_FA) ? 1 : 0;
    tstart(c, GF_K_FFT_XY_FWD);
    hipLaunchKernelGGL((k_fft_xy<T, kEPT, false>), dim3(gridA), dim3(L.thrA), L.ldsA, c->st, Z, L.ps, L.n[0], L.n[1],
                       nzt, L.G, L.rs, c->plan[0], c->plan[1], tw[0], tw[1], c->ctl, force);
    tstop(c);
    tstart(c, GF_K_FFT_ZT);
    hipLaunchKernelGGL((k_fft_zt<T, kEPT>), dim3(gridB), dim3(L.thrB), L.ldsB, c->st, Z, L.ps, L.n[0], L.n[1],
                       L.n[2], L.n[3], L.bx, L.tsp, c->plan[2], c->plan[3], tw[2], tw[3],
                       reinterpret_cast<const T*>(c->sin2), (T)coef, no_fa, c->ctl, force);
    tstop(c);
    tstart(c, GF_K_FFT_XY_INV);
    hipLaunchKernelGGL((k_fft_xy<T, kEPT, true>), dim3(gridA), dim3(L.thrA), L.ldsA, c->st, Z, L.ps, L.n[0], L.n[1],
                       nzt, L.G, L.rs, c->plan[0], c->plan[1], tw[0], tw[1], c->ctl, force);
    tstop(c);
    return check_hip(c, hipGetLastError(), "fft launch");
}

template <typename T, int NE>
gf_status launch_measure_t(gf_ctx* c, int force) {
    const Layout& L = c->L;
    tstart(c, GF_K_DIVERGENCE);
    hipLaunchKernelGGL((k_divergence<T, NE>), dim3(L.nblk), dim3(kSiteThreads), 0, c->st, links_of<T, NE>(c),
                       reinterpret_cast<cx<T>*>(c->Z), L.ps, c->geom, c->part, c->ctl, force);
    tstop(c);
    tstart(c, GF_K_FINALIZE);
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(256), 0, c->st, c->part, L.nblk, 1.0 / (3.0 * (double)L.vol),
                       1.0 / (12.0 * (double)L.vol), c->ctl, force);
    tstop(c);
    return check_hip(c, hipGetLastError(), "divergence launch");
}

template <typename T, int NE>
gf_status launch_update_t(gf_ctx* c, int count) {
    const Layout& L = c->L;
    tstart(c, GF_K_UPDATE);
    hipLaunchKernelGGL((k_update<T, NE>), dim3(L.nblk), dim3(kSiteThreads), 0, c->st, links_of<T, NE>(c),
                       reinterpret_cast<const cx<T>*>(c->Z), L.ps, c->geom, c->ctl, count);
    tstop(c);
    return check_hip(c, hipGetLastError(), "update launch");
}

#define GF_DISPATCH(c, fn, ...)                                                   \
    ((c)->L.fp32 ? ((c)->L.ne == 6 ? fn<float, 6>(__VA_ARGS__) : fn<float, 9>(__VA_ARGS__)) \
                 : ((c)->L.ne == 6 ? fn<double, 6>(__VA_ARGS__) : fn<double, 9>(__VA_ARGS__)))

gf_status launch_measure(gf_ctx* c, int force) { return GF_DISPATCH(c, launch_measure_t, c, force); }
gf_status launch_update(gf_ctx* c, int count) { return GF_DISPATCH(c, launch_update_t, c, count); }
gf_status launch_fft_any(gf_ctx* c, int force) {
    return c->L.fp32 ? launch_fft<float>(c, force) : launch_fft<double>(c, force);
}

template <typename T, int NE>
gf_status launch_pack_t(gf_ctx* c, const double* src) {
    const int reunit = sizeof(T) == 4 ? 1 : 0;
    hipLaunchKernelGGL((k_pack<T, NE>), dim3(c->L.nblk), dim3(kSiteThreads), 0, c->st, src, links_of<T, NE>(c),
                       c->L.vol, reunit);
    return check_hip(c, hipGetLastError(), "pack launch");
}
template <typename T, int NE>
gf_status launch_unpack_t(gf_ctx* c, double* dst) {
    hipLaunchKernelGGL((k_unpack<T, NE>), dim3(c->L.nblk), dim3(kSiteThreads), 0, c->st, links_of<T, NE>(c), dst,
                       c->L.vol);
    return check_hip(c, hipGetLastError(), "unpack launch");
}

gf_status read_head(gf_ctx* c) {
    GF_TRY_HIP(c, hipMemcpyAsync(c->h_head, c->ctl, kHeadBytes, hipMemcpyDeviceToHost, c->st));
    GF_TRY_HIP(c, hipStreamSynchronize(c->st));
    if (c->npend) tdrain(c);
    return GF_OK;
}

gf_status set_tol(gf_ctx* c, double tol) {
    hipLaunchKernelGGL(k_set_tol, dim3(1), dim3(64), 0, c->st, c->ctl, tol);
    return check_hip(c, hipGetLastError(), "set_tol launch");
}

gf_status one_iteration(gf_ctx* c) {
    gf_status s = launch_fft_any(c, 0);
    if (s == GF_OK) s = launch_update(c, 1);
    if (s == GF_OK) s = launch_measure(c, 0);
    return s;
}

// FFT kernels may take more than 64 KB of dynamic LDS (gfx950 has 160 KB per CU).
void raise_lds_limits() {
    static bool done = false;
    if (done) return;
    const int cap = 160 * 1024;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_xy<double, kEPT, false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_xy<double, kEPT, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_zt<double, kEPT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_xy<float, kEPT, false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_xy<float, kEPT, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_zt<float, kEPT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipGetLastError();
    done = true;
}

template <typename T>
void fill_tables(gf_ctx* c, std::vector<unsigned char>& host) {
    // sin^2 table: [Nx | Ny | Nz | Nt] values of 4 sin^2(pi n / N); twiddles W_N^k per axis.
    const Layout& L = c->L;
    host.assign(L.off_z - L.off_sin2, 0);
    T* s2 = reinterpret_cast<T*>(host.data());
    int k = 0;
    for (int d = 0; d < 4; ++d)
        for (int n = 0; n < L.n[d]; ++n) {
            const long double sv = sinl(3.14159265358979323846264338327950288L * (long double)n / (long double)L.n[d]);
            s2[k++] = (T)(4.0L * sv * sv);
        }
    for (int d = 0; d < 4; ++d) {
        cx<T>* tw = reinterpret_cast<cx<T>*>(host.data() + (L.off_tw - L.off_sin2) + (size_t)d * kMaxExtent * 16);
        for (int n = 0; n < L.n[d]; ++n) {
            const long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)n / (long double)L.n[d];
            tw[n] = {(T)cosl(a), (T)sinl(a)};
        }
    }
}

template <typename T>
void field_pack(gf_ctx* c, const void* src, double scale) {
    hipLaunchKernelGGL(k_field_pack<T>, dim3(c->L.nblk), dim3(kSiteThreads), 0, c->st,
                       reinterpret_cast<const double*>(src), reinterpret_cast<cx<T>*>(c->Z), c->L.ps, c->L.vol, scale);
}
template <typename T>
void field_unpack(gf_ctx* c, void* dst) {
    hipLaunchKernelGGL(k_field_unpack<T>, dim3(c->L.nblk), dim3(kSiteThreads), 0, c->st,
                       reinterpret_cast<const cx<T>*>(c->Z), c->L.ps, reinterpret_cast<double*>(dst), c->L.vol);
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
        c->Z = c->ws + L.off_z;
        c->links = c->ws + L.off_links;
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
        // Tables.
        std::vector<unsigned char> host;
        if (L.fp32)
            fill_tables<float>(c, host);
        else
            fill_tables<double>(c, host);
        Ctl head{};
        head.tol = -1.0;
        auto done_fail = [&](gf_status st) {
            g_init_error = c->err;
            (void)hipHostFree(c->h_head);
            delete c;
            return st;
        };
        if ((s = check_hip(c, hipMemcpyAsync(c->sin2, host.data(), host.size(), hipMemcpyHostToDevice, c->st),
                           "table upload")) != GF_OK)
            return done_fail(s);
        if ((s = check_hip(c, hipMemcpyAsync(c->ctl, &head, kHeadBytes, hipMemcpyHostToDevice, c->st),
                           "control upload")) != GF_OK)
            return done_fail(s);
        const double* src = c->links_user;
        s = GF_DISPATCH(c, launch_pack_t, c, src);
        if (s == GF_OK) s = launch_measure(c, 1);
        if (s == GF_OK) s = read_head(c);
        if (s != GF_OK) return done_fail(s);
        *out = c;
        return GF_OK;
    } catch (...) {
        g_init_error = "unexpected host exception";
        return GF_EINVAL;
    }
}

static gf_status run_loop(gf_ctx* c, double tol, int64_t max_iter, gf_result* r) {
    const auto t0 = std::chrono::steady_clock::now();
    gf_status s = set_tol(c, tol);
    if (s == GF_OK) s = read_head(c);
    if (s != GF_OK) return s;
    const long long start = c->h_head->iters;
    while (!c->h_head->done && c->h_head->iters - start < max_iter) {
        const int64_t left = max_iter - (c->h_head->iters - start);
        const int64_t k = std::min<int64_t>(left, c->p.check_every);
        for (int64_t i = 0; i < k && s == GF_OK; ++i) s = one_iteration(c);
        if (s == GF_OK) s = read_head(c);
        if (s != GF_OK) return s;
    }
    s = GF_DISPATCH(c, launch_unpack_t, c, c->links_user);
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
    if (!c || !theta || !F) return c ? fail(c, GF_EINVAL, "null output") : GF_EINVAL;
    gf_status s = read_head(c);
    if (s != GF_OK) return s;
    *theta = c->h_head->theta;
    *F = c->h_head->F;
    return GF_OK;
}

gf_status gf_get_links(gf_ctx* c, void* d_out) {
    if (!c) return GF_EINVAL;
    if (!d_out) return fail(c, GF_EINVAL, "d_out is NULL");
    gf_status s = GF_DISPATCH(c, launch_unpack_t, c, reinterpret_cast<double*>(d_out));
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
    gf_status s = launch_measure(c, 1);
    if (s != GF_OK) return s;
    if (c->L.fp32)
        hipLaunchKernelGGL(k_field_unpack<float>, dim3(c->L.nblk), dim3(kSiteThreads), 0, c->st,
                           reinterpret_cast<const cx<float>*>(c->Z), c->L.ps, reinterpret_cast<double*>(d_delta),
                           c->L.vol);
    else
        hipLaunchKernelGGL(k_field_unpack<double>, dim3(c->L.nblk), dim3(kSiteThreads), 0, c->st,
                           reinterpret_cast<const cx<double>*>(c->Z), c->L.ps, reinterpret_cast<double*>(d_delta),
                           c->L.vol);
    GF_TRY_HIP(c, hipGetLastError());
    return read_head(c);
}

gf_status gf_stage_filter(gf_ctx* c, const void* d_in, void* d_out) {
    if (!c) return GF_EINVAL;
    if (!d_in || !d_out) return fail(c, GF_EINVAL, "null pointer");
    if (c->L.fp32) field_pack<float>(c, d_in, 1.0); else field_pack<double>(c, d_in, 1.0);
    GF_TRY_HIP(c, hipGetLastError());
    gf_status s = launch_fft_any(c, 1);
    if (s != GF_OK) return s;
    if (c->L.fp32) field_unpack<float>(c, d_out); else field_unpack<double>(c, d_out);
    GF_TRY_HIP(c, hipGetLastError());
    return check_hip(c, hipStreamSynchronize(c->st), "sync");
}

gf_status gf_stage_update(gf_ctx* c, const void* d_scaled) {
    if (!c) return GF_EINVAL;
    if (!d_scaled) return fail(c, GF_EINVAL, "null pointer");
    if (c->L.fp32) field_pack<float>(c, d_scaled, 1.0); else field_pack<double>(c, d_scaled, 1.0);
    GF_TRY_HIP(c, hipGetLastError());
    // Run the update regardless of the stop flag, without counting it.
    gf_status s = set_tol(c, -1.0);
    if (s == GF_OK) s = launch_update(c, 0);
    if (s == GF_OK) s = GF_DISPATCH(c, launch_unpack_t, c, c->links_user);
    if (s != GF_OK) return s;
    return check_hip(c, hipStreamSynchronize(c->st), "sync");
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
    if (c->h_head) (void)hipHostFree(c->h_head);
    for (auto& e : c->ev) (void)hipEventDestroy(e);
    delete c;
}

}  // extern "C"

// libgf host side of the temporal Wilson-line singlet correlator (gf_wilson_* in include/gf.h).
//
// The handle carves the caller's workspace into: the nine Wilson-line element
// planes (transformed in place), the spectrum S, a correlator table used when
// the caller passes none, the x/y/z twiddle tables and the shell lists (offsets
// and members, each shell's members in increasing site order). Tables are
// uploaded once at creation; every later call only queues kernels on the stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/gf.h"
#include "gf_wilson.hpp"

using namespace gf;

struct gf_wilson {
    int n[4];
    int vs;
    size_t wps;  // complex elements per Wilson-line plane
    int chunks;  // t chunks per spatial site in k_wilson_lines
    int rs;      // padded row length of an (x, y) plane in LDS
    int bx;      // in-plane positions per k_wcorr_z block
    int thr_xy, thr_z;
    size_t lds_xy, lds_z;
    FftPlan px, py, pz;
    int nshell;
    std::vector<int> r2, count;
    cx<double>* W;
    cx<double>* S;
    double* corr;
    cx<double>* tw[3];
    int* off;
    int* members;
    hipStream_t st;
    std::string err;
};

namespace {

constexpr int kWEpt = 4;  // FFT elements per thread per stage (small blocks of short work: more waves)
constexpr int kWMaxExtent = 64;
constexpr size_t kWAlign = 256;

thread_local std::string g_wilson_error;

size_t walign(size_t x) { return (x + kWAlign - 1) / kWAlign * kWAlign; }
int wround64(int x) { return (x + 63) / 64 * 64; }

bool w_is_2a3b(int n) {
    if (n < 1) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

// Radix sequence: threes, then eights and fours, a two if left (the order the Stockham stages expect).
FftPlan w_plan(int n) {
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

struct WLayout {
    int n[4];
    int vs;
    size_t wps;
    int nshell;
    size_t off_W, off_S, off_corr, off_tw[3], off_off, off_mem, total;
};

gf_status w_layout(const int32_t* dims, WLayout& L, std::string& err) {
    if (!dims) {
        err = "dims is NULL";
        return GF_EINVAL;
    }
    int64_t vs = 1;
    for (int i = 0; i < 4; ++i) {
        const int n = dims[i];
        if (n < 2) {
            err = "every extent must be >= 2";
            return GF_EINVAL;
        }
        if (n % 2 != 0 || !w_is_2a3b(n) || n > kWMaxExtent) {
            err = "extent " + std::to_string(n) + " unsupported: each extent must be even, of the form 2^a 3^b and <= " +
                  std::to_string(kWMaxExtent);
            return GF_ENOTSUP;
        }
        L.n[i] = n;
        if (i < 3) vs *= n;
    }
    L.vs = (int)vs;
    L.wps = (size_t)(vs + 63) / 64 * 64;
    // shells: distinct minimum-image r^2 (at most sum_i (N_i/2)^2 + 1 of them)
    std::vector<char> seen(3 * (kWMaxExtent / 2) * (kWMaxExtent / 2) + 1, 0);
    int ns = 0;
    for (int a = 0; a <= L.n[0] / 2; ++a)
        for (int b = 0; b <= L.n[1] / 2; ++b)
            for (int c = 0; c <= L.n[2] / 2; ++c) {
                const int r2 = a * a + b * b + c * c;
                if (!seen[r2]) {
                    seen[r2] = 1;
                    ++ns;
                }
            }
    L.nshell = ns;
    size_t o = 0;
    L.off_W = o;
    o = walign(o + 9 * L.wps * sizeof(cx<double>));
    L.off_S = o;
    o = walign(o + L.wps * sizeof(cx<double>));
    L.off_corr = o;
    o = walign(o + L.wps * sizeof(double));
    for (int d = 0; d < 3; ++d) {
        L.off_tw[d] = o;
        o = walign(o + L.n[d] * sizeof(cx<double>));
    }
    L.off_off = o;
    o = walign(o + (size_t)(ns + 1) * sizeof(int));
    L.off_mem = o;
    o = walign(o + (size_t)vs * sizeof(int));
    L.total = o;
    return GF_OK;
}

gf_status wfail(gf_wilson* w, gf_status s, const std::string& msg) {
    if (w) w->err = msg;
    return s;
}

gf_status wcheck(gf_wilson* w, hipError_t e, const char* what) {
    if (e == hipSuccess) return GF_OK;
    return wfail(w, GF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void raise_wilson_lds() {
    static bool done = false;
    if (done) return;
    const int cap = 160 * 1024;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_wcorr_xy_fwd<kWEpt>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_wcorr_xy_inv<kWEpt>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_wcorr_z<kWEpt>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    done = true;
}

template <int C, int STRIDE>
void launch_lines(gf_wilson* w, const double* links, double* lines) {
    hipLaunchKernelGGL((k_wilson_lines<C, STRIDE>), dim3((w->vs + kWlSites - 1) / kWlSites), dim3(64 * C), 0, w->st,
                       reinterpret_cast<const double2*>(links), w->vs, w->n[3], w->W, w->wps,
                       reinterpret_cast<double2*>(lines));
}

template <int STRIDE>
void launch_lines_c(gf_wilson* w, const double* links, double* lines) {
    if (w->chunks == 8)
        launch_lines<8, STRIDE>(w, links, lines);
    else if (w->chunks == 4)
        launch_lines<4, STRIDE>(w, links, lines);
    else
        launch_lines<2, STRIDE>(w, links, lines);
}

gf_status correlator(gf_wilson* w, const double* d_links, bool temporal_only, double* d_lines, double* d_corr,
                     double* d_shell);

}  // namespace

extern "C" {

size_t gf_wilson_workspace_bytes(const int32_t* dims) {
    WLayout L;
    std::string err;
    return w_layout(dims, L, err) == GF_OK ? L.total : 0;
}

gf_status gf_wilson_create(gf_wilson** out, const int32_t* dims, void* d_workspace, size_t workspace_bytes,
                           void* stream) {
    if (!out) {
        g_wilson_error = "out is NULL";
        return GF_EINVAL;
    }
    *out = nullptr;
    WLayout L;
    std::string err;
    gf_status s = w_layout(dims, L, err);
    if (s != GF_OK) {
        g_wilson_error = err;
        return s;
    }
    if (!d_workspace || workspace_bytes < L.total) {
        g_wilson_error = "workspace is NULL or smaller than gf_wilson_workspace_bytes";
        return GF_EINVAL;
    }
    if (reinterpret_cast<uintptr_t>(d_workspace) % kWAlign) {
        g_wilson_error = "workspace must be 256-byte aligned";
        return GF_EINVAL;
    }
    gf_wilson* w = new (std::nothrow) gf_wilson();
    if (!w) {
        g_wilson_error = "out of host memory";
        return GF_EINVAL;
    }
    for (int i = 0; i < 4; ++i) w->n[i] = L.n[i];
    w->vs = L.vs;
    w->wps = L.wps;
    w->st = reinterpret_cast<hipStream_t>(stream);
    unsigned char* ws = static_cast<unsigned char*>(d_workspace);
    w->W = reinterpret_cast<cx<double>*>(ws + L.off_W);
    w->S = reinterpret_cast<cx<double>*>(ws + L.off_S);
    w->corr = reinterpret_cast<double*>(ws + L.off_corr);
    for (int d = 0; d < 3; ++d) w->tw[d] = reinterpret_cast<cx<double>*>(ws + L.off_tw[d]);
    w->off = reinterpret_cast<int*>(ws + L.off_off);
    w->members = reinterpret_cast<int*>(ws + L.off_mem);
    const int nx = L.n[0], ny = L.n[1], nz = L.n[2], nt = L.n[3];
    // t chunks per site: as many as divide Nt while each chunk keeps two links or more (one in flight
    // while the other is multiplied), at most 8
    w->chunks = 2;
    for (int c : {8, 4})
        if (nt % c == 0 && nt / c >= 2) {
            w->chunks = c;
            break;
        }
    w->px = w_plan(nx);
    w->py = w_plan(ny);
    w->pz = w_plan(nz);
    w->rs = nx + 1;  // odd row stride: the y transform's columns fall in different LDS banks
    w->thr_xy = std::min(1024, std::max(64, wround64((nx * ny + kWEpt - 1) / kWEpt)));
    w->lds_xy = (size_t)(nx + ny + (size_t)w->rs * ny) * sizeof(cx<double>);
    const int plane = nx * ny;
    w->bx = 4;  // 64-byte runs per z row; the plane (both extents even) always divides
    (void)plane;
    w->thr_z = std::min(1024, std::max(64, wround64((9 * w->bx * nz + kWEpt - 1) / kWEpt)));
    w->lds_z = (size_t)(nz + (size_t)10 * w->bx * nz) * sizeof(cx<double>);
    // host tables: twiddles, shells (ordered by r^2, members by site index)
    const long double pi = 3.14159265358979323846264338327950288L;
    std::vector<cx<double>> tw[3];
    for (int d = 0; d < 3; ++d) {
        tw[d].resize(L.n[d]);
        for (int k = 0; k < L.n[d]; ++k) {
            const long double a = -2.0L * pi * (long double)k / (long double)L.n[d];
            tw[d][k] = {(double)cosl(a), (double)sinl(a)};
        }
    }
    std::map<int, std::vector<int>> shells;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const int a = std::min(x, nx - x), b = std::min(y, ny - y), c = std::min(z, nz - z);
                shells[a * a + b * b + c * c].push_back(x + nx * (y + ny * z));
            }
    w->nshell = (int)shells.size();
    std::vector<int> off, mem;
    off.reserve(w->nshell + 1);
    mem.reserve(w->vs);
    for (auto& kv : shells) {
        off.push_back((int)mem.size());
        w->r2.push_back(kv.first);
        w->count.push_back((int)kv.second.size());
        mem.insert(mem.end(), kv.second.begin(), kv.second.end());
    }
    off.push_back((int)mem.size());
    raise_wilson_lds();
    for (int d = 0; d < 3 && s == GF_OK; ++d)
        s = wcheck(w, hipMemcpyAsync(w->tw[d], tw[d].data(), tw[d].size() * sizeof(cx<double>),
                                     hipMemcpyHostToDevice, w->st),
                   "twiddle upload");
    if (s == GF_OK)
        s = wcheck(w, hipMemcpyAsync(w->off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice, w->st),
                   "shell upload");
    if (s == GF_OK)
        s = wcheck(w, hipMemcpyAsync(w->members, mem.data(), mem.size() * sizeof(int), hipMemcpyHostToDevice, w->st),
                   "shell upload");
    // the host vectors go away on return: wait for the copies
    const gf_status sync = wcheck(w, hipStreamSynchronize(w->st), "sync");
    if (s == GF_OK) s = sync;
    if (s != GF_OK) {
        g_wilson_error = w->err;
        delete w;
        return s;
    }
    *out = w;
    return GF_OK;
}

int32_t gf_wilson_shell_count(const gf_wilson* w) { return w ? w->nshell : -1; }

gf_status gf_wilson_shells(const gf_wilson* w, int32_t* h_r2, int32_t* h_count) {
    if (!w) return GF_EINVAL;
    for (int s = 0; s < w->nshell; ++s) {
        if (h_r2) h_r2[s] = w->r2[s];
        if (h_count) h_count[s] = w->count[s];
    }
    return GF_OK;
}

gf_status gf_wilson_correlator(gf_wilson* w, const double* d_links, double* d_lines, double* d_corr,
                               double* d_shell) {
    if (!w) return GF_EINVAL;
    if (!d_links) return wfail(w, GF_EINVAL, "d_links is NULL");
    return correlator(w, d_links, false, d_lines, d_corr, d_shell);
}

gf_status gf_wilson_correlator_temporal(gf_wilson* w, const double* d_temporal, double* d_lines, double* d_corr,
                                        double* d_shell) {
    if (!w) return GF_EINVAL;
    if (!d_temporal) return wfail(w, GF_EINVAL, "d_temporal is NULL");
    return correlator(w, d_temporal, true, d_lines, d_corr, d_shell);
}

}  // extern "C"

namespace {

gf_status correlator(gf_wilson* w, const double* d_links, bool temporal_only, double* d_lines, double* d_corr,
                     double* d_shell) {
    const int nx = w->n[0], ny = w->n[1], nz = w->n[2];
    double* corr = d_corr ? d_corr : w->corr;
    if (temporal_only)
        launch_lines_c<9>(w, d_links, d_lines);
    else
        launch_lines_c<36>(w, d_links, d_lines);
    gf_status s = wcheck(w, hipGetLastError(), "wilson lines launch");
    if (s != GF_OK) return s;
    hipLaunchKernelGGL(k_wcorr_xy_fwd<kWEpt>, dim3(nz, 9), dim3(w->thr_xy), w->lds_xy, w->st, w->W, w->wps, nx, ny,
                       w->rs, w->px, w->py, w->tw[0], w->tw[1]);
    if ((s = wcheck(w, hipGetLastError(), "xy forward launch")) != GF_OK) return s;
    hipLaunchKernelGGL(k_wcorr_z<kWEpt>, dim3(nx * ny / w->bx), dim3(w->thr_z), w->lds_z, w->st, w->W, w->wps,
                       nx * ny, nz, w->bx, w->pz, w->tw[2], w->S);
    if ((s = wcheck(w, hipGetLastError(), "z pass launch")) != GF_OK) return s;
    const double vs = (double)w->vs;
    hipLaunchKernelGGL(k_wcorr_xy_inv<kWEpt>, dim3(nz), dim3(w->thr_xy), w->lds_xy, w->st, w->S, nx, ny, w->rs,
                       w->px, w->py, w->tw[0], w->tw[1], 1.0 / (3.0 * vs * vs), corr);
    if ((s = wcheck(w, hipGetLastError(), "xy inverse launch")) != GF_OK) return s;
    if (d_shell) {
        hipLaunchKernelGGL(k_wcorr_shells, dim3((w->nshell + 3) / 4), dim3(256), 0, w->st, corr, w->off, w->members,
                           w->nshell, d_shell);
        if ((s = wcheck(w, hipGetLastError(), "shell launch")) != GF_OK) return s;
    }
    return GF_OK;
}

}  // namespace

extern "C" {

const char* gf_wilson_last_error(const gf_wilson* w) { return w ? w->err.c_str() : g_wilson_error.c_str(); }

void gf_wilson_destroy(gf_wilson* w) {
    if (!w) return;
    (void)hipStreamSynchronize(w->st);
    delete w;
}

}  // extern "C"

// libgf host side of the Monte Carlo input generator (gf_mc_* in include/gf.h).
//
// The handle keeps the lattice shape, beta, the seed and a workspace of the
// caller's: the even/odd link planes the sweeps run on (72 planes of V/2
// complex doubles), per-block counters of rejected heatbath pair updates,
// plaquette partials and two result scalars. A call packs the canonical links
// into the planes, runs its sweeps (8 launches per heatbath or over-relaxation
// pass: 4 directions x 2 parities; then one reunitarisation launch) and
// unpacks; all on the handle's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>

#include "../../include/gf.h"
#include "gf_mc.hpp"

using namespace gf;

struct gf_mc {
    McGeom g;
    McPlanes P;
    double beta;
    unsigned long long seed;
    int nblk_half;  // blocks of one (mu, parity) launch
    int nblk_plaq;
    unsigned* rej;
    double* part;
    unsigned long long* d_count;
    double* d_plaq;
    hipStream_t st;
    std::string err;
};

namespace {

constexpr int kMcMaxExtent = 256;
constexpr size_t kMcAlign = 256;

thread_local std::string g_mc_error;

size_t mc_align(size_t x) { return (x + kMcAlign - 1) / kMcAlign * kMcAlign; }

struct McLayout {
    McGeom g;
    int nblk_half, nblk_plaq;
    size_t hp;
    size_t off_planes, off_rej, off_part, off_count, off_plaq, total;
};

gf_status mc_layout(const int32_t* dims, McLayout& L, std::string& err) {
    if (!dims) {
        err = "dims is NULL";
        return GF_EINVAL;
    }
    long long vol = 1;
    for (int i = 0; i < 4; ++i) {
        const int n = dims[i];
        if (n < 2 || n % 2 != 0) {
            err = "every extent must be even and >= 2 (even/odd site updates)";
            return GF_EINVAL;
        }
        if (n > kMcMaxExtent) {
            err = "extent " + std::to_string(n) + " above " + std::to_string(kMcMaxExtent);
            return GF_ENOTSUP;
        }
        L.g.n[i] = n;
        vol *= n;
    }
    if (vol * 4 > 0xFFFFFFFFll) {
        err = "more than 2^32 links (the link index is one 32-bit counter word)";
        return GF_ENOTSUP;
    }
    L.g.vol = vol;
    L.g.half_x = L.g.n[0] / 2;
    L.nblk_half = (int)((vol / 2 + kMcThreads - 1) / kMcThreads);
    L.nblk_plaq = (int)((vol + 255) / 256);
    L.hp = (size_t)(vol / 2 + 255) / 256 * 256;
    size_t o = 0;
    L.off_planes = o;
    o = mc_align(o + 72 * L.hp * sizeof(double2));
    L.off_rej = o;
    o = mc_align(o + (size_t)L.nblk_half * sizeof(unsigned));
    L.off_part = o;
    o = mc_align(o + (size_t)L.nblk_plaq * sizeof(double));
    L.off_count = o;
    o = mc_align(o + sizeof(unsigned long long));
    L.off_plaq = o;
    o = mc_align(o + sizeof(double));
    L.total = o;
    return GF_OK;
}

gf_status mfail(gf_mc* m, gf_status s, const std::string& msg) {
    if (m) m->err = msg;
    return s;
}

gf_status mcheck(gf_mc* m, hipError_t e, const char* what) {
    if (e == hipSuccess) return GF_OK;
    return mfail(m, GF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

McKey make_key(const gf_mc* m, unsigned word1, unsigned purpose) {
    return {(unsigned)(m->seed & 0xFFFFFFFFull), (unsigned)(m->seed >> 32), word1, purpose};
}

}  // namespace

extern "C" {

size_t gf_mc_workspace_bytes(const int32_t* dims) {
    McLayout L;
    std::string err;
    return mc_layout(dims, L, err) == GF_OK ? L.total : 0;
}

gf_status gf_mc_create(gf_mc** out, const int32_t* dims, double beta, uint64_t seed, void* d_workspace,
                       size_t workspace_bytes, void* stream) {
    if (!out) {
        g_mc_error = "out is NULL";
        return GF_EINVAL;
    }
    *out = nullptr;
    McLayout L;
    std::string err;
    gf_status s = mc_layout(dims, L, err);
    if (s != GF_OK) {
        g_mc_error = err;
        return s;
    }
    if (!(beta > 0.0) || !std::isfinite(beta)) {
        g_mc_error = "beta must be positive and finite";
        return GF_EINVAL;
    }
    if (!d_workspace || workspace_bytes < L.total || reinterpret_cast<uintptr_t>(d_workspace) % kMcAlign) {
        g_mc_error = "workspace is NULL, not 256-byte aligned or smaller than gf_mc_workspace_bytes";
        return GF_EINVAL;
    }
    gf_mc* m = new (std::nothrow) gf_mc();
    if (!m) {
        g_mc_error = "out of host memory";
        return GF_EINVAL;
    }
    m->g = L.g;
    m->beta = beta;
    m->seed = seed;
    m->nblk_half = L.nblk_half;
    m->nblk_plaq = L.nblk_plaq;
    unsigned char* ws = static_cast<unsigned char*>(d_workspace);
    m->P = {reinterpret_cast<double2*>(ws + L.off_planes), L.hp};
    m->rej = reinterpret_cast<unsigned*>(ws + L.off_rej);
    m->part = reinterpret_cast<double*>(ws + L.off_part);
    m->d_count = reinterpret_cast<unsigned long long*>(ws + L.off_count);
    m->d_plaq = reinterpret_cast<double*>(ws + L.off_plaq);
    m->st = reinterpret_cast<hipStream_t>(stream);
    *out = m;
    return GF_OK;
}

gf_status gf_mc_update(gf_mc* m, double* d_links, uint64_t first_sweep, int32_t n_sweeps, int32_t n_overrelax,
                       int64_t* h_rejected) {
    if (!m) return GF_EINVAL;
    if (!d_links) return mfail(m, GF_EINVAL, "d_links is NULL");
    if (n_sweeps < 1) return mfail(m, GF_EINVAL, "n_sweeps must be >= 1");
    if (first_sweep + (uint64_t)n_sweeps - 1 > 0xFFFFFFFFull) return mfail(m, GF_EINVAL, "sweeps must fit in 32 bits");
    if (n_overrelax < 0 || n_overrelax > 64) return mfail(m, GF_EINVAL, "n_overrelax must be in [0, 64]");
    double2* links = reinterpret_cast<double2*>(d_links);
    const unsigned nsite_blk = (unsigned)((m->g.vol + 255) / 256);
    hipLaunchKernelGGL(k_mc_zero, dim3((m->nblk_half + 255) / 256), dim3(256), 0, m->st, m->rej, m->nblk_half);
    gf_status s = mcheck(m, hipGetLastError(), "counter reset launch");
    if (s != GF_OK) return s;
    hipLaunchKernelGGL(k_mc_pack, dim3(nsite_blk), dim3(256), 0, m->st, links, m->P, m->g);
    if ((s = mcheck(m, hipGetLastError(), "pack launch")) != GF_OK) return s;
    const long long half = m->g.vol / 2;
    for (int32_t k = 0; k < n_sweeps && s == GF_OK; ++k) {
        const McKey key = make_key(m, (unsigned)(first_sweep + k), 0);
        for (int rep = 0; rep <= n_overrelax && s == GF_OK; ++rep)
            for (int mu = 0; mu < 4 && s == GF_OK; ++mu)
                for (int par = 0; par < 2 && s == GF_OK; ++par) {
                    if (rep == 0)
                        hipLaunchKernelGGL(k_mc_update<false>, dim3(m->nblk_half), dim3(kMcThreads), 0, m->st, m->P,
                                           m->g, mu, par, m->beta, key, m->rej);
                    else
                        hipLaunchKernelGGL(k_mc_update<true>, dim3(m->nblk_half), dim3(kMcThreads), 0, m->st, m->P,
                                           m->g, mu, par, m->beta, key, m->rej);
                    s = mcheck(m, hipGetLastError(), "update launch");
                }
        if (s != GF_OK) return s;
        hipLaunchKernelGGL(k_mc_reunit, dim3((unsigned)((8 * half + 255) / 256)), dim3(256), 0, m->st, m->P, half);
        s = mcheck(m, hipGetLastError(), "reunitarisation launch");
    }
    if (s != GF_OK) return s;
    hipLaunchKernelGGL(k_mc_unpack, dim3(nsite_blk), dim3(256), 0, m->st, m->P, m->g, links);
    if ((s = mcheck(m, hipGetLastError(), "unpack launch")) != GF_OK) return s;
    if (h_rejected) {
        hipLaunchKernelGGL(k_mc_count, dim3(1), dim3(256), 0, m->st, m->rej, m->nblk_half, m->d_count);
        if ((s = mcheck(m, hipGetLastError(), "count launch")) != GF_OK) return s;
        unsigned long long v = 0;
        if ((s = mcheck(m, hipMemcpyAsync(&v, m->d_count, sizeof(v), hipMemcpyDeviceToHost, m->st), "readback")) !=
            GF_OK)
            return s;
        if ((s = mcheck(m, hipStreamSynchronize(m->st), "sync")) != GF_OK) return s;
        *h_rejected = (int64_t)v;
    }
    return GF_OK;
}

gf_status gf_mc_multihit(gf_mc* m, const double* d_links, uint64_t tag, int32_t n_hits, double* d_out) {
    if (!m) return GF_EINVAL;
    if (!d_links || !d_out) return mfail(m, GF_EINVAL, "d_links or d_out is NULL");
    if (tag > 0xFFFFFFFFull) return mfail(m, GF_EINVAL, "tag must fit in 32 bits");
    if (n_hits < 1 || n_hits > 4095) return mfail(m, GF_EINVAL, "n_hits must be in [1, 4095]");
    hipLaunchKernelGGL(k_mc_multihit, dim3((unsigned)((m->g.vol + kMcThreads - 1) / kMcThreads)), dim3(kMcThreads), 0,
                       m->st, reinterpret_cast<const double2*>(d_links), m->g, m->beta, make_key(m, (unsigned)tag, 1),
                       n_hits, reinterpret_cast<double2*>(d_out));
    return mcheck(m, hipGetLastError(), "multi-hit launch");
}

gf_status gf_mc_plaquette(gf_mc* m, const double* d_links, double* h_plaquette) {
    if (!m) return GF_EINVAL;
    if (!d_links || !h_plaquette) return mfail(m, GF_EINVAL, "d_links or h_plaquette is NULL");
    hipLaunchKernelGGL(k_mc_plaquette, dim3(m->nblk_plaq), dim3(256), 0, m->st,
                       reinterpret_cast<const double2*>(d_links), m->g, m->part);
    gf_status s = mcheck(m, hipGetLastError(), "plaquette launch");
    if (s != GF_OK) return s;
    hipLaunchKernelGGL(k_mc_plaquette_sum, dim3(1), dim3(256), 0, m->st, m->part, m->nblk_plaq,
                       1.0 / (18.0 * (double)m->g.vol), m->d_plaq);
    if ((s = mcheck(m, hipGetLastError(), "plaquette sum launch")) != GF_OK) return s;
    double v = 0.0;
    if ((s = mcheck(m, hipMemcpyAsync(&v, m->d_plaq, sizeof(v), hipMemcpyDeviceToHost, m->st), "readback")) != GF_OK)
        return s;
    if ((s = mcheck(m, hipStreamSynchronize(m->st), "sync")) != GF_OK) return s;
    *h_plaquette = v;
    return GF_OK;
}

const char* gf_mc_last_error(const gf_mc* m) { return m ? m->err.c_str() : g_mc_error.c_str(); }

void gf_mc_destroy(gf_mc* m) {
    if (!m) return;
    (void)hipStreamSynchronize(m->st);
    delete m;
}

}  // extern "C"

// One launch per pass over every configuration of a batch of uneven lattices.
//
// A batch of independent configurations of several shapes runs each step of the iteration as one
// launch: the blocks of all active configurations form one grid, each block finds its configuration by
// a binary search in a table of first blocks (one entry per active configuration, rebuilt by the host
// when the active set changes), reads its lattice's parameters from a per-shape table in device memory
// and runs the runtime-shaped body of the pass on that configuration's slab. No block waits for another
// and the kernel boundaries order the passes, as in the single-lattice loop.
#pragma once

#include "gf_kernels.hpp"

namespace gf {

constexpr int kMaxFusedGroups = 8;

// The parameters of one lattice shape of a batch (configuration 0 of the shape; configuration c's
// buffers are c*cs bytes further on). Written once by the host when the batch is set up.
template <typename T>
struct FusedGroup {
    size_t cs;
    Ctl* ctl;
    double2* part;
    const cx<T>* U0;
    cx<T>* D;
    cx<T>* Q;
    cx<T>* H[2];
    const T* sin2;
    const cx<T>* tw[4];
    size_t ps;
    Geom geom;
    FftPlan plan[4];
    int G, rs, bx, tsp;
    int npart;  // loop-kernel partials per configuration
    double coef, inv3v, inv12v;
    int blocks[4];  // blocks per configuration of the (x, y), (z, t), gauge and loop passes
};

// The active configurations of one launch: segment j is configuration cfg[j] of shape group[j]; its
// blocks of pass p are first[p][j] .. first[p][j + 1] - 1.
struct FusedTable {
    const int* first[4];
    const int* group;
    const int* cfg;
    int nseg;
};

// Segment of global block b (first[0] = 0, first[nseg] = the grid size).
__device__ __forceinline__ int fused_segment(const int* __restrict__ first, int nseg, int b) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename P>
__device__ __forceinline__ P* fshift(P* p, size_t o) {
    return reinterpret_cast<P*>(reinterpret_cast<uintptr_t>(p) + o);
}

// (x, y) forward pass D -> Q of every active configuration; the first block of each configuration also
// reduces that configuration's pending loop partials.
template <typename T, int EPT>
__global__ void __launch_bounds__(1024) k_fused_xy(const FusedGroup<T>* __restrict__ grp, FusedTable tb) {
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int j = fused_segment(tb.first[0], tb.nseg, b);
    const FusedGroup<T>& g = grp[tb.group[j]];
    const size_t o = (size_t)tb.cfg[j] * g.cs;
    const int local = b - tb.first[0][j];
    fft_xy_body<T, EPT, false>(fshift(g.D, o), fshift(g.Q, o), g.ps, g.geom.n[0], g.geom.n[1],
                               g.geom.n[2] * g.geom.n[3], g.G, g.rs, g.plan[0], g.plan[1], fshift(g.tw[0], o),
                               fshift(g.tw[1], o), fshift(g.ctl, o), 0, fshift(g.part, o), g.npart, g.inv3v, g.inv12v,
                               local, local == 0);
}

// (z, t) forward pass, filter and inverse, in Q.
template <typename T, int EPT>
__global__ void __launch_bounds__(1024) k_fused_zt(const FusedGroup<T>* __restrict__ grp, FusedTable tb, int no_fa) {
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int j = fused_segment(tb.first[1], tb.nseg, b);
    const FusedGroup<T>& g = grp[tb.group[j]];
    const size_t o = (size_t)tb.cfg[j] * g.cs;
    TupleGeom tg{};
    fft_zt_body<T, EPT>(fshift(g.Q, o), g.ps, g.geom.n[0], g.geom.n[1], g.geom.n[2], g.geom.n[3], g.bx, g.tsp,
                        g.plan[2], g.plan[3], fshift(g.tw[2], o), fshift(g.tw[3], o), fshift(g.sin2, o), (T)g.coef,
                        no_fa, fshift(g.ctl, o), 0, nullptr, tg, nullptr, b - tb.first[1][j]);
}

// Inverse (x, y) pass, g and the update H[hp] -> H[1 - hp]. NTMAX: the block size bound (512 when every
// shape's planes take at most 512 threads, which leaves the double-precision body its registers).
template <typename T, int EPT, int NTMAX>
__global__ void __launch_bounds__(NTMAX) k_fused_gauge(const FusedGroup<T>* __restrict__ grp, FusedTable tb, int hp,
                                                      int exact) {
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int j = fused_segment(tb.first[2], tb.nseg, b);
    const FusedGroup<T>& g = grp[tb.group[j]];
    const size_t o = (size_t)tb.cfg[j] * g.cs;
    fft_xy_gauge_body<T, EPT>(fshift(g.Q, o), g.ps, fshift(g.H[hp], o), fshift(g.H[1 - hp], o), g.geom.n[0],
                              g.geom.n[1], g.rs, g.plan[0], g.plan[1], fshift(g.tw[0], o), fshift(g.tw[1], o),
                              fshift(g.ctl, o), 0, exact, b - tb.first[2][j]);
}

// Loop kernel (one block per 64-site block, the plain sweep) on the links H[hp] U0 H[hp]^dag.
template <typename T, int NE>
__global__ void __launch_bounds__(kFusedThreads, 2) k_fused_loop(const FusedGroup<T>* __restrict__ grp, FusedTable tb,
                                                                 int hp) {
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int j = fused_segment(tb.first[3], tb.nseg, b);
    const FusedGroup<T>& g = grp[tb.group[j]];
    const size_t o = (size_t)tb.cfg[j] * g.cs;
    Ctl* ctl = fshift(g.ctl, o);
    if (ctl->done) return;
    const LoopIO<T, NE> io{Links<T, NE>{const_cast<cx<T>*>(fshift(g.U0, o)), g.ps}, fshift(g.H[hp], o),
                           fshift(g.D, o), g.ps};
    const int sb = b - tb.first[3][j];
    const int lane = threadIdx.x & 63;
    const int mu = lane >> 4;
    const int64_t s = (int64_t)sb * kFusedSites + (threadIdx.x >> 6) * 16 + (lane & 15);
    double fsum, tsum;
    loop_site_block<T, NE, false>(io, g.geom, s, s < g.geom.vol, mu, false, nullptr, fsum, tsum);
    if (threadIdx.x == 0) {
        fshift(g.part, o)[sb] = make_double2(fsum, tsum);
        if (sb == 0) ctl->pending = 1;
    }
}

// The pending loop partials of every active configuration, one block each.
template <typename T>
__global__ void __launch_bounds__(256) k_fused_finalize(const FusedGroup<T>* __restrict__ grp, FusedTable tb) {
    const int j = blockIdx.x;
    const FusedGroup<T>& g = grp[tb.group[j]];
    const size_t o = (size_t)tb.cfg[j] * g.cs;
    Ctl* ctl = fshift(g.ctl, o);
    if (!ctl->pending) return;
    reduce_partials(fshift(g.part, o), g.npart, g.inv3v, g.inv12v, ctl, 1);
}

}  // namespace gf

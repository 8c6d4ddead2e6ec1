/*
 * gf.h - C ABI of libgf, Landau gauge fixing of SU(3) lattice gauge fields by
 * Fourier-accelerated steepest descent on one AMD MI355X (gfx950).
 *
 * The problem (paper, Section 1): given links U_mu(x) in SU(3) on a periodic
 * 4D lattice, find a gauge transform g(x) that maximises the Landau functional
 *     F = 1/(4*3*V) sum_x sum_mu Re Tr U_mu(x)
 * by steepest descent with Fourier acceleration (Davies et al. 1988). One
 * iteration computes the lattice divergence
 *     Delta(x) = M - M^dag - (1/3) Tr(M - M^dag),  M = sum_mu [U_mu(x-mu) - U_mu(x)],
 * filters it in momentum space by p2max/p^2 (Section 2.2: every matrix element
 * is transformed separately; the 4D FFT is split 2D + 2D), forms
 *     g(x) = reunitarize(1 + (alpha/2) Delta~(x))
 * and applies U_mu(x) -> g(x) U_mu(x) g(x+mu)^dag. Quality:
 *     theta = 1/(3V) sum_x Tr[Delta Delta^dag].
 * Links may be stored with all 18 reals or with the first two rows only
 * (12 reals; the third row is rebuilt from unitarity, Section 2.2).
 *
 * Layouts. dims = {Nx, Ny, Nz, Nt}; site s = x + Nx*(y + Ny*(z + Nz*t)).
 * "Canonical links" are complex double (re, im interleaved) in the order
 * [s][mu][row][col], i.e. 4*9 complex per site, mu = 0..3 for x, y, z, t.
 * "Canonical matrix field" is complex double [s][row][col].
 *
 * Ownership. The caller owns every device buffer (links, workspace, outputs);
 * libgf allocates no device memory. The context is a small host object. All
 * device work is queued on the caller's stream; calls that return scalars
 * synchronise that stream. Pointers named d_* are device pointers.
 *
 * Errors. Every call returns a gf_status and never throws. GF_EINVAL and
 * GF_ENOTSUP leave every buffer untouched. GF_ENOTCONV: the iteration limit
 * was reached; links hold the last iterate and the result is filled in.
 * GF_ENUMERIC: theta is NaN or infinite. GF_EDEVICE: a HIP call failed
 * (gf_last_error gives the HIP message).
 */
#ifndef GF_H
#define GF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gf_ctx gf_ctx;

typedef enum {
    GF_OK = 0,
    GF_EINVAL = 1,    /* bad argument (null pointer, bad size, tol <= 0, ...) */
    GF_ENOTSUP = 2,   /* valid but unsupported (extent not even or not 2^a 3^b, too large) */
    GF_EDEVICE = 3,   /* HIP runtime error */
    GF_ENOTCONV = 4,  /* max_iter reached before theta < tol */
    GF_ENUMERIC = 5,  /* theta not finite */
    GF_ESTATE = 6     /* call not valid in the context's current state */
} gf_status;

/* Link storage and arithmetic precision of the bulk iterations. */
typedef enum {
    GF_FP64_18 = 0,   /* double, full 3x3 matrix */
    GF_FP64_12 = 1,   /* double, rows 1-2, row 3 rebuilt on every read */
    GF_FP32_12 = 2,   /* float, rows 1-2 (re-orthonormalised on write) */
    GF_FP32_18 = 3,   /* float, full matrix */
    GF_MIXED = 4      /* FP32-12 until theta < switch_theta, then FP64-18; the hand-over comes
                         earlier if the float descent stalls: no new minimum of theta for 200
                         updates while theta < 1e-6, or for 2000 at any theta */
} gf_precision;

enum {
    GF_FLAG_EXACT_EXP = 1u << 0,   /* g = reunitarize(exp((alpha/2) Delta~)) (closed-form SU(3) exponential,
                                      Cayley-Hamilton) instead of reunitarize(1 + (alpha/2) Delta~) */
    GF_FLAG_NO_FA = 1u << 1,       /* plain steepest descent: K(p) = 1 instead of p2max/p^2 */
    GF_FLAG_GENERIC_FFT = 1u << 2, /* use the runtime-shaped FFT kernels even where a compile-time one exists */
    GF_FLAG_ACCUMULATE_GAUGE = 1u << 3, /* accepted and ignored: the accumulated transform G(x) with
                                           U = G U_input G(x+mu)^dag is what every context stores (gf_get_gauge) */
    GF_FLAG_LEARNED = 1u << 4,          /* reserve the learned preconditioner (gf_mlp_set_weights) */
    GF_FLAG_RECORD_SPECTRA = 1u << 5,   /* reserve spectrum recording (gf_record_spectra) */
    GF_FLAG_BATCH_FUSED = 1u << 6       /* batches: every pass of an iteration is one launch over all active
                                           configurations of every shape (runtime-shaped FFT kernels, the plain
                                           loop sweep); single contexts: the same kernels, so that a single
                                           solve and a fused batch give the same bits */
};

typedef struct {
    int32_t dims[4];       /* Nx, Ny, Nz, Nt: each even, >= 2, of the form 2^a 3^b, <= 64 */
    int32_t precision;     /* gf_precision */
    double alpha;          /* step size (0.08 in the reference workloads) */
    double switch_theta;   /* GF_MIXED: theta at which FP32 hands over to FP64 (1e-8) */
    int32_t check_every;   /* host reads theta every this many iterations (>= 1) */
    uint32_t flags;        /* GF_FLAG_* */
} gf_params;

typedef struct {
    int64_t iters;         /* updates applied since gf_init */
    double theta;          /* quality of the current links */
    double F;              /* functional of the current links */
    int32_t phase;         /* 0: FP32 bulk (GF_MIXED only), 1: FP64 */
    int32_t fallbacks;     /* GF_FLAG_LEARNED: learned updates rejected by the device guard and
                              replaced by a plain FA update (0 otherwise) */
    double seconds;        /* wall time of the call */
} gf_result;

/* Bytes of device workspace gf_init needs for these parameters (0 if invalid). */
size_t gf_workspace_bytes(const gf_params* params);

/*
 * Create a context. d_links: canonical links (V*36 complex double), read now
 * and overwritten with the current iterate at the end of every gf_iterate /
 * gf_fix_until. d_workspace: >= gf_workspace_bytes(params) bytes, 256-byte
 * aligned, owned by the caller and untouched by it while the context lives.
 * stream: a hipStream_t (NULL = default stream). Measures theta and F of the
 * input before returning.
 */
gf_status gf_init(gf_ctx** ctx, const gf_params* params, void* d_links,
                  void* d_workspace, size_t workspace_bytes, void* stream);

/* Apply exactly n >= 0 updates (no stopping test); result holds theta, F after them. */
gf_status gf_iterate(gf_ctx* ctx, int64_t n, gf_result* result);

/*
 * gf_iterate without the egress: exactly n >= 0 updates (Section 1: one FA iteration each), leaving the
 * links in the context's working layout; the caller's d_links are NOT written. gf_get_links(ctx, d_links)
 * writes them out, and so does the next gf_iterate or gf_fix_until. For callers that only read theta and
 * F between calls (and for timing the iteration itself). Plain contexts only: GF_MIXED and batch
 * contexts return GF_ESTATE and change nothing.
 */
gf_status gf_advance(gf_ctx* ctx, int64_t n, gf_result* result);

/*
 * Iterate until theta < theta_tol (theta measured before each update), or
 * until max_iter updates have been applied in this call (GF_ENOTCONV).
 */
gf_status gf_fix_until(gf_ctx* ctx, double theta_tol, int64_t max_iter, gf_result* result);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): gf_init + gf_fix_until + gf_destroy in one call, with the
 * workspace taken from the library's own device-resident scratch instead of a caller buffer.
 * The scratch is a file-scope device array of GF_NOALLOC_SCRATCH_BYTES (128 MiB) per GPU, held from the
 * first call on that GPU until the process ends; the call allocates no device memory and calls no HIP
 * allocation routine (the small context object lives on the host heap for the duration of the call).
 * d_links: canonical links (V*36 complex double), read and overwritten with the result (on GF_ENOTCONV
 * with the last iterate). stream: hipStream_t (NULL = default stream); the call synchronises it.
 * GF_ENOTSUP (nothing touched) if gf_workspace_bytes(params) exceeds the scratch: up to 16^4 in every
 * precision, 32^3 x 4 in FP64-12 or FP32-12. Every call on one GPU shares its scratch: calls that overlap
 * on the same GPU (other host threads, other streams) race and must be serialised by the caller.
 * gf_last_error(NULL) describes a failure.
 */
#define GF_NOALLOC_SCRATCH_BYTES (128ull << 20)
gf_status gf_fix_until_noalloc(const gf_params* params, void* d_links, void* stream, double theta_tol,
                               int64_t max_iter, gf_result* result);

/*
 * Batches of independent lattices (many uneven configurations, one GPU).
 * The gauge fixing of Section 1 of the paper acts on each configuration on
 * its own (the paper fixes one lattice at a time); a batch advances every configuration of the same
 * shape in the same kernel launches, each with its own stopping test, and
 * retires a configuration as soon as its theta < theta_tol. params: n sets
 * that may differ in dims only (precision, alpha, switch_theta, check_every
 * and flags equal; GF_FLAG_LEARNED and GF_FLAG_RECORD_SPECTRA not allowed).
 * GF_MIXED configurations iterate in float until theta < switch_theta (or the
 * float descent stalls) and finish in double precision, as in gf_init.
 * Without GF_FLAG_BATCH_FUSED each shape group runs its own launches (the
 * compile-time FFT kernels of its shape) on a stream of its own; with it, all
 * shapes advance together on the caller's stream and each pass of an
 * iteration is one launch over every active configuration (at most 8 shapes,
 * x-y planes of at most 2048 sites; GF_ENOTSUP otherwise), the phases of
 * GF_MIXED in step. The fused passes run the runtime-shaped FFT bodies: a
 * configuration ends bitwise equal to a single context created with the same
 * flags (GF_FLAG_BATCH_FUSED on a single context selects those bodies too).
 */

/* Bytes of device workspace gf_init_batch needs (0 if the parameters are invalid). */
size_t gf_batch_workspace_bytes(int32_t n, const gf_params* params);

/*
 * Create a batch context. d_links[i]: canonical links of configuration i
 * (V_i*36 complex double, device), read now and overwritten with the final
 * iterate by gf_fix_until_batch. d_workspace: >= gf_batch_workspace_bytes
 * bytes, 256-byte aligned, caller-owned. Measures theta and F of every input.
 * A batch context takes only gf_fix_until_batch, gf_last_error and
 * gf_destroy (GF_ESTATE otherwise).
 */
gf_status gf_init_batch(gf_ctx** ctx, int32_t n, const gf_params* params, double* const* d_links,
                        void* d_workspace, size_t workspace_bytes, void* stream);

/*
 * Fix every configuration to theta < theta_tol, each within max_iter updates
 * (float and double phases counted together). results[i] (host, n entries)
 * receives configuration i's outcome; seconds is the wall time of the whole
 * call. Returns GF_ENOTCONV (or GF_ENUMERIC) if any configuration failed;
 * results and links are filled in for all of them.
 */
gf_status gf_fix_until_batch(gf_ctx* ctx, double theta_tol, int64_t max_iter, gf_result* results);

/*
 * FFT tiling in use (for GF_MIXED: of the active phase): planes per block of
 * the (x, y) passes and x columns per block of the (z, t) pass. gf_init picks
 * them by timing the compile-time alternatives for the lattice shape and
 * precision, once per process (GF_FLAG_GENERIC_FFT: the runtime-shaped
 * kernels' defaults).
 */
gf_status gf_fft_tiling(gf_ctx* ctx, int32_t* xy_planes, int32_t* zt_columns);

/*
 * Override the FFT tiling of this context (a test and measurement aid): one of
 * the compile-time alternatives for the lattice shape and precision, which
 * compute the same transforms. GF_EINVAL if the pair is not one of them (the
 * message lists the planes and columns compiled for the shape), GF_ESTATE
 * under GF_FLAG_GENERIC_FFT or for a batch context. For GF_MIXED: the active
 * phase.
 */
gf_status gf_set_fft_tiling(gf_ctx* ctx, int32_t xy_planes, int32_t zt_columns);

/*
 * Traversal of the loop kernel (update + divergence + theta/F partials).
 * z_group >= 1: blocks of 64 sites sweep the (x, y) planes, taking z in groups
 * of z_group planes inside the t loop, so that t neighbours are still cached.
 * z_group == 0 (t-march): each block owns 64 sites of the (x, y, z) volume and
 * steps through t, keeping its own updated U_t of one step for the divergence
 * of the next, so U_t(x - t) and g(x - t) are not fetched again.
 * z_group == -1 (brick march): each block owns a brick of whole x rows (by rows
 * in y, bz planes in z, Nx*by a multiple of 64) and steps through a segment of
 * t; every link is formed once, by the lane that owns it, and the divergence
 * takes the back links from LDS (from a halo lane where the back neighbour lies
 * outside the brick). gf_init times the traversals that fit the shape (1; 2, 4,
 * 8 where they divide Nz and 64 divides Nx*Ny; 0 where 64 divides Nx*Ny*Nz,
 * Nt >= 4 and there are >= 32 blocks; -1 where a divisor by of Ny makes Nx*by a
 * multiple of 64 with 4*Nx*by <= 1024 and the link arrays stay below 4 GiB) on
 * the first context of a shape and precision in the process and keeps the
 * fastest. Partials are summed by site block, so every traversal
 * gives bitwise the same results. gf_set_loop_traversal overrides the choice for
 * this context (a test and measurement aid); GF_EINVAL if z_group is not one
 * of the candidates. For GF_MIXED: the active phase.
 */
gf_status gf_loop_traversal(gf_ctx* ctx, int32_t* z_group);
gf_status gf_set_loop_traversal(gf_ctx* ctx, int32_t z_group);

/*
 * Mean plaquette of the current links, (1/(18V)) sum_x sum_{mu<nu} Re Tr[
 * U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag], summed in double precision
 * in a fixed order. Gauge invariant: gauge fixing must leave it unchanged
 * (the check of a result without the input's gauge).
 */
gf_status gf_plaquette(gf_ctx* ctx, double* plaquette);

/* theta and F of the current links, in double precision. */
gf_status gf_quality(gf_ctx* ctx, double* theta, double* F);

/* Write the current links to d_out in canonical layout (d_out may be the input buffer). */
gf_status gf_get_links(gf_ctx* ctx, void* d_out);

/*
 * Write the accumulated gauge transform G (canonical matrix field, V*9
 * complex double) with U_current(x) = G(x) U_input(x) G(x+mu)^dag. Every
 * context keeps G (it stores the links in this form: the input links and G,
 * rows 1-2, which every update replaces by reunitarize(g G), the
 * re-orthonormalisation in double precision in every precision).
 */
gf_status gf_get_gauge(gf_ctx* ctx, void* d_out);

/*
 * Checkpoint and resume. gf_get_state writes the complete state of a context
 * (links, iteration count, theta/F history, precision phase, accumulated
 * gauge, network parameters) to the device buffer d_out of at least
 * gf_state_bytes(ctx) bytes; gf_set_state restores it into a context created
 * with the same gf_params (else GF_EINVAL, nothing changed) and writes the
 * restored links to that context's d_links. Continuing after a restore gives
 * bitwise the same iterates as never stopping. The buffer is opaque and is
 * only meant for the same build of libgf. Not for batch contexts (0 bytes,
 * GF_ESTATE).
 */
size_t gf_state_bytes(const gf_ctx* ctx);
gf_status gf_get_state(gf_ctx* ctx, void* d_out, size_t bytes);
gf_status gf_set_state(gf_ctx* ctx, const void* d_in, size_t bytes);

/*
 * Copy the last n recorded (theta_k, F_k) pairs, k = iters-n+1 .. iters, into
 * host arrays (n <= 16384 and n <= iters + 1). GF_MIXED: the history of the
 * active phase, counted from the start of that phase.
 */
gf_status gf_history(gf_ctx* ctx, int64_t n, double* h_theta, double* h_F);

/*
 * Single-stage entry points (used to check each step separately; they do not
 * advance the iteration count).
 *   gf_stage_divergence: Delta(x) of the current links -> d_delta (canonical
 *     matrix field); also refreshes theta and F.
 *   gf_stage_filter: d_in (canonical anti-Hermitian traceless field) ->
 *     d_out = (alpha/2) * IFFT[K(p) FFT[d_in]] (canonical matrix field).
 *   gf_stage_gauge: d_in as for gf_stage_filter -> d_out = g(x) =
 *     reunitarize(1 + (alpha/2) Delta~(x)) (canonical matrix field; with
 *     GF_FLAG_EXACT_EXP of exp((alpha/2) Delta~(x))), the gauge transform the
 *     loop applies.
 *   gf_stage_update: U_mu(x) -> g U_mu(x) g(x+mu)^dag with
 *     g = reunitarize(1 + d_scaled(x)) (GF_FLAG_EXACT_EXP: of exp(d_scaled(x))),
 *     d_scaled a canonical field that already holds (alpha/2) Delta~.
 */
gf_status gf_stage_divergence(gf_ctx* ctx, void* d_delta);
gf_status gf_stage_filter(gf_ctx* ctx, const void* d_in, void* d_out);
gf_status gf_stage_gauge(gf_ctx* ctx, const void* d_in, void* d_out);
gf_status gf_stage_update(gf_ctx* ctx, const void* d_scaled);

/*
 * Per-kernel timing with HIP events recorded on the context's stream around
 * kernel launches. gf_set_timing(ctx, 1) resets the totals and times every
 * kernel (0 stops); gf_set_timing_mask(ctx, mask) times only the kernel ids
 * whose bit (1 << GF_K_*) is set, so that the others run without events in
 * between. gf_kernel_times copies, for kernel ids 0..n-1 (GF_K_*), the summed
 * duration in milliseconds and the number of launches timed.
 */
enum {
    GF_K_FFT_XY_FWD = 0,  /* forward 2D FFT over (x, y) */
    GF_K_FFT_ZT = 1,      /* 2D FFT over (z, t), filter, inverse (z, t) */
    GF_K_FFT_XY_INV = 2,  /* inverse 2D FFT over (x, y) (in the loop: followed by g(x)) */
    GF_K_UPDATE = 3,      /* single-stage update U_mu(x) -> g(x) U_mu(x) g(x+mu)^dag */
    GF_K_DIVERGENCE = 4,  /* standalone Delta(x) and block partial sums of F, theta */
    GF_K_FINALIZE = 5,    /* fixed-order reduction -> theta, F, stop flag */
    GF_K_UPDATE_MEASURE = 6,  /* loop kernel: update, divergence of the new links, reduction */
    GF_NKERNELS = 8
};
gf_status gf_set_timing(gf_ctx* ctx, int32_t enable);
gf_status gf_set_timing_mask(gf_ctx* ctx, uint32_t mask);
gf_status gf_kernel_times(gf_ctx* ctx, int32_t n, double* h_ms_total, int64_t* h_counts);

/*
 * Learned spectral preconditioner (an extension of the paper's fixed filter).
 * The multiplier of mode p becomes m0(p) exp(o_s(p) + o_a(0)), where m0 is
 * the Fourier-acceleration multiplier (alpha/2) p2max/p^2 and (o_s, o_a) are
 * the outputs of a 6 -> 64 -> 64 -> 2 tanh network (float) on the features
 * of the momentum tuple n_mu in [0, N_mu/2] at iteration k:
 *   x = (p^2_mu/4 - 1/2 for mu = 0..3, log10(theta_k)/8 + 1, k/64),
 * o_a being read at the zero tuple. Parameters, gf_mlp_param_count() floats:
 * W1 (64x6, row-major), b1 (64), W2 (64x64), b2 (64), W3 (2x64), b3 (2).
 * A learned step that increases theta, lowers F (beyond 1e-14) or gives a
 * theta that is not finite is stopped on the device, undone and replaced by a
 * plain Fourier-accelerated step; after its r-th such rejection the network
 * pauses for 2^r plain steps, and after 6 it stays off (gf_result.fallbacks
 * counts the rejections).
 */
int32_t gf_mlp_param_count(void);

/* Copy d_params (device) into the context and switch the network on (enable = 1) or off. */
gf_status gf_mlp_set_weights(gf_ctx* ctx, const float* d_params, int32_t enable);

/*
 * Write the multiplier table the network gives at the current theta and
 * iteration count to d_out (device; T entries over the folded tuples, first
 * axis fastest; double for FP64 contexts, float for FP32):
 * d_out[i] = (alpha/2) p2max / (V p^2_i) * exp(o_s(i) + o_a(0)), 0 at the zero
 * tuple, the 1/V of the inverse FFT included. Needs GF_FLAG_LEARNED.
 */
gf_status gf_mlp_multipliers(gf_ctx* ctx, void* d_out);

/*
 * Apply n plain Fourier-accelerated updates and record, for every step k and
 * every momentum tuple i (n_mu in [0, N_mu/2], first axis fastest), summed
 * over the tuple's +-n reflections and the four packed divergence fields
 * after the forward FFT (T tuples, double):
 *   d_records[(k*T + i)*3 + 0] = P_k = sum |Z_k(p)|^2,
 *   [.. + 1] = C_k = sum Re[Z_{k+1}(p) conj(Z_k(p))],
 *   [.. + 2] = E_k = sum |Z'_k(p)|^2, Z' the divergence after a probe update
 *              from step k with every multiplier times probe_scale (in (0, 1)),
 *              which is then undone.
 * h_theta[k] = theta_k. Needs GF_FLAG_RECORD_SPECTRA; the network is not used.
 */
gf_status gf_record_spectra(gf_ctx* ctx, int64_t n, double probe_scale, double* d_records, double* h_theta);

/*
 * Training (no lattice context). Rows are momentum tuples of samples; sample
 * s owns rows [offsets[s], offsets[s+1]) of x (6 floats per row, the features
 * above) and tgt (a, b, c per row, from gf_mlp_make_samples), its first row
 * being the zero tuple. With s(p) = exp(o_s(p) + o_a(first row)) the factor
 * on the plain multiplier, the predicted residual energy ratio of a sample
 * after the scaled step is R = sum_p e_p(s_p) / sum_p a = sum_p (a - 2 s b +
 * s^2 c) / sum_p a; its loss
 * is ln(max(R, 1e-12)) (zero gradient below), and the loss is the mean over
 * samples: the predicted mean log-decrease per step. All pointers are device pointers except
 * h_loss (host, may be NULL); d_ws holds gf_mlp_workspace_bytes(n_rows,
 * n_samples) bytes. Adam: beta1 0.9, beta2 0.999, eps 1e-8, step from 1.
 */
size_t gf_mlp_workspace_bytes(int64_t n_rows, int32_t n_samples);
/*
 * Training rows from n_records consecutive records of gf_record_spectra made
 * with probe_scale sigma (d_theta[r] = theta of record r, iteration k0 + r).
 * Sample s uses record r = first + s*every and record r + 1 (so
 * r <= n_records - 2, else GF_EINVAL): row s*T + i of d_x gets the features
 * of tuple i at (theta_r, k0 + r), and of d_tgt (a, b, c), the coefficients
 * of the quadratic e(x) = a - 2 b x + c x^2 through the residual energies of
 * the mode after the step scaled by x: e(0) = P_r, e(sigma) = E_r,
 * e(1) = P_{r+1} (c raised to b^2/a where needed, so that e >= 0).
 * dims: host array {Nx, Ny, Nz, Nt}; T = prod(N_mu/2 + 1).
 */
gf_status gf_mlp_make_samples(const double* d_records, int32_t n_records, const double* d_theta,
                              int32_t first, int32_t every, int32_t n_samples, int64_t k0,
                              double probe_scale, const int32_t* dims, float* d_x, float* d_tgt,
                              void* stream);
gf_status gf_mlp_forward(const float* d_params, const float* d_x, int64_t n_rows, float* d_out,
                         void* d_ws, size_t ws_bytes, void* stream);
gf_status gf_mlp_loss_grad(const float* d_params, const float* d_x, const float* d_tgt,
                           const int32_t* d_offsets, int32_t n_samples, int64_t n_rows, float* d_grad,
                           void* d_ws, size_t ws_bytes, void* stream, double* h_loss);
gf_status gf_mlp_adam(float* d_params, float* d_m, float* d_v, const float* d_grad, int64_t step,
                      float lr, void* stream);
gf_status gf_mlp_train_step(float* d_params, float* d_m, float* d_v, int64_t step, float lr,
                            const float* d_x, const float* d_tgt, const int32_t* d_offsets,
                            int32_t n_samples, int64_t n_rows, float* d_grad, void* d_ws,
                            size_t ws_bytes, void* stream, double* h_loss);

/* Message of the last error on this context (or of the last failed gf_init if ctx is NULL). */
const char* gf_last_error(const gf_ctx* ctx);

/* Free the host context (the caller frees its own device buffers). */
void gf_destroy(gf_ctx* ctx);

/*
 * Measurement aid, not part of the method: a plain streaming copy of `bytes`
 * (a multiple of 16; both pointers 16-byte aligned, device, caller-owned, not
 * overlapping) queued on stream, 16 bytes per lane with nontemporal loads and
 * stores. It gives the device bandwidth on the simplest read-once/write-once
 * traffic, against which the kernels' bandwidth figures are read.
 */
gf_status gf_stream_copy(const void* d_src, void* d_dst, size_t bytes, void* stream);

/* ------------------------------------------------------------------------
 * Temporal Wilson lines and the colour-singlet correlator (paper, Section 1,
 * Eq. (1)): the singlet free energy comes from (1/3) < Tr W(r) W(0)^dag >,
 * which is not gauge invariant and is taken on the Landau-gauge-fixed field.
 * For one configuration:
 *     W(x) = U_t(x, 0) U_t(x, 1) ... U_t(x, Nt-1)          (x spatial)
 *     C(r) = 1/(3 Vs) sum_x Re Tr[W(x + r) W(x)^dag]       (every r, periodic)
 * with Vs = Nx Ny Nz; the ensemble average over configurations is the
 * caller's. The imaginary part is odd in r and is dropped (it cancels in any
 * average over r and -r). Shells group the separations by the minimum-image
 * r^2 = sum_i min(r_i, N_i - r_i)^2, in increasing r^2; a shell's value is
 * the mean of C over its members, summed in a fixed order. The sum over x
 * runs as a cyclic correlation by 3D FFT of the nine matrix elements.
 * Double precision throughout. dims as in gf_params (each extent even,
 * 2^a 3^b, <= 64).
 * ---------------------------------------------------------------------- */
typedef struct gf_wilson gf_wilson;

/* Device workspace bytes for these dims (0 if invalid). */
size_t gf_wilson_workspace_bytes(const int32_t dims[4]);

/*
 * Create a handle over the caller's workspace (>= gf_wilson_workspace_bytes,
 * 256-byte aligned, owned by the caller and kept for the handle's life).
 * Uploads the twiddle and shell tables on stream (a hipStream_t, NULL = the
 * default stream) and synchronises it. GF_EINVAL / GF_ENOTSUP: nothing is
 * created (gf_wilson_last_error(NULL) gives the reason).
 */
gf_status gf_wilson_create(gf_wilson** out, const int32_t dims[4], void* d_workspace,
                           size_t workspace_bytes, void* stream);

/* Number of shells (-1 for a NULL handle). */
int32_t gf_wilson_shell_count(const gf_wilson* w);

/* Host copies of each shell's r^2 and member count (either pointer may be NULL). */
gf_status gf_wilson_shells(const gf_wilson* w, int32_t* h_r2, int32_t* h_count);

/*
 * Queue the correlator of canonical links d_links (complex double
 * [s][mu][row][col], the layout gf_init takes and returns) on the handle's
 * stream; nothing is synchronised. Outputs (device, caller-owned; each may be
 * NULL): d_lines, W as complex double [xs][row][col] with xs = x + Nx(y + Ny z);
 * d_corr, C(r) as double [rz][ry][rx]; d_shell, gf_wilson_shell_count doubles.
 * Calls on one handle must not overlap (they share its workspace).
 */
gf_status gf_wilson_correlator(gf_wilson* w, const double* d_links, double* d_lines, double* d_corr,
                               double* d_shell);

/*
 * The same from a field of temporal links alone, complex double [s][row][col]
 * (V x 9), e.g. the multi-hit averages of gf_mc_multihit (which need not be
 * unitary): W(x) is the ordered product of these matrices along t.
 */
gf_status gf_wilson_correlator_temporal(gf_wilson* w, const double* d_temporal, double* d_lines, double* d_corr,
                                        double* d_shell);

/* Message of the last error on this handle (or of the last failed create if w is NULL). */
const char* gf_wilson_last_error(const gf_wilson* w);

/* Free the handle (synchronises its stream first). */
void gf_wilson_destroy(gf_wilson* w);

/* ------------------------------------------------------------------------
 * Monte Carlo input generator. The paper gauge-fixes thermalised SU(3)
 * configurations (Section 3: 32^4 at beta = 5.8, 6.0, 6.2) and applies
 * multi-hit to the temporal links before fixing (Section 1), without
 * stating either algorithm; these are the standard ones:
 *   Wilson action S = beta sum_p (1 - (1/3) Re Tr U_p); the link U_mu(x) has
 *   local weight exp((beta/3) Re Tr(U A)), A the sum of its six staples.
 *   Heatbath: Cabibbo-Marinari over the SU(2) subgroups of rows (0,1), (0,2),
 *   (1,2), each drawn by Kennedy-Pendleton. Over-relaxation: the SU(2)
 *   reflection that keeps Re Tr(U A). A sweep updates the 4 directions, even
 *   sites then odd, and reunitarises every link at the end.
 *   Multi-hit: with all other links fixed, the average of n successive
 *   heatbath updates of each temporal link (not reunitarised).
 * Random numbers are Philox4x32-10 (Salmon et al., SC11) keyed by the seed,
 * with counters (link index 4s + mu, sweep or tag, hit/pair/draw, purpose),
 * so results depend only on (seed, sweep/tag) and not on the launch shape.
 * Links are canonical (see gf_init), updated in place. Every extent even and
 * in [2, 256]; at most 2^32 links. Double precision throughout.
 * ---------------------------------------------------------------------- */
typedef struct gf_mc gf_mc;

/* Device workspace bytes for these dims (0 if invalid). */
size_t gf_mc_workspace_bytes(const int32_t dims[4]);

/*
 * Create a generator handle: beta > 0 and finite, any 64-bit seed, workspace
 * >= gf_mc_workspace_bytes (about 576 B per site: the even/odd copy of the
 * links) and 256-byte aligned (caller-owned, kept for the handle's life),
 * stream a hipStream_t (NULL = default). Queues nothing.
 * GF_EINVAL / GF_ENOTSUP: nothing created (gf_mc_last_error(NULL)).
 */
gf_status gf_mc_create(gf_mc** out, const int32_t dims[4], double beta, uint64_t seed, void* d_workspace,
                       size_t workspace_bytes, void* stream);

/*
 * n_sweeps (>= 1) sweeps in place on d_links; sweep k (k = first_sweep ..
 * first_sweep + n_sweeps - 1, all < 2^32) is one heatbath sweep with the
 * random numbers of k, then n_overrelax (0..64) over-relaxation sweeps, then
 * every link reunitarised. The links are packed into the handle's even/odd
 * planes once before the first sweep and written back after the last. If
 * h_rejected is not NULL the stream is synchronised and it receives the
 * number of SU(2) pair updates that kept their old value because 64
 * Kennedy-Pendleton attempts were all rejected (the chain then stays where it
 * was, which keeps the target distribution; 0 in practice at beta >~ 1).
 * Otherwise nothing is synchronised.
 */
gf_status gf_mc_update(gf_mc* m, double* d_links, uint64_t first_sweep, int32_t n_sweeps, int32_t n_overrelax,
                       int64_t* h_rejected);

/*
 * Multi-hit average of every temporal link with the random numbers of `tag`
 * (< 2^32) and n_hits (1..4095) hits: d_out is complex double [s][row][col]
 * (V x 9, caller-owned); d_links is only read. Queued, not synchronised.
 */
gf_status gf_mc_multihit(gf_mc* m, const double* d_links, uint64_t tag, int32_t n_hits, double* d_out);

/* Mean plaquette (1/(18V)) sum Re Tr U_p of canonical links, fixed-order FP64 sum; synchronises. */
gf_status gf_mc_plaquette(gf_mc* m, const double* d_links, double* h_plaquette);

/* Message of the last error on this handle (or of the last failed create if m is NULL). */
const char* gf_mc_last_error(const gf_mc* m);

/* Free the handle (synchronises its stream first). */
void gf_mc_destroy(gf_mc* m);

#ifdef __cplusplus
}
#endif

#endif /* GF_H */

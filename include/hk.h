/*
 * hk.h -- C ABI of libhk, the MI355X (gfx950) implementation of the hot path of hypothesis-tested
 * progressive kernel estimation ("Hypothesis Testing for Progressive Kernel Estimation and VCM
 * Framework", arXiv 2504.04411).
 *
 * One iteration (Sec. 5.1) for every hit point (kernel, eye vertex):
 *   1. sort the iteration's light vertices (photons) into a uniform grid (counting/radix sort by cell),
 *   2. gather the photons inside the kernel's current radius r (Eq. kaplanyan-integral, disk Omega_r),
 *   3. map each one to the kernel's tangent plane (Eq. map-function) and add its test sample to the
 *      sums and sums of squares of its group: 2 equi-areal annuli x 6 equi-angular sectors
 *      (Sec. 3.2.1, Sec. 6.1.1), retained while the radius is kept (Sec. 5.1),
 *   4. evaluate the ANOVA F statistic (Eq. f-statistic) against the (1 - alpha_F) quantile of
 *      F(11, 12 (m - 1)) (Sec. 3.2.2), m = light sub-paths since the last shrink,
 *   5. add this iteration's kernel estimate to the progressive estimate (Eq. progressive-VCM-estimator)
 *      and shrink the radius when the test rejects (Eq. radiusupdate),
 *   6. in vertex-merging mode, weight each merged pair by the balance heuristic (Eq. mis-weight).
 *
 * Conventions
 *   - Every call returns an int status: HK_OK (0) or a negative HK_E_* code; hk_last_error() gives a
 *     message for the calling thread. No call aborts the process.
 *   - Calls taking a hipStream_t only enqueue work on that stream; they do not synchronise (except
 *     where stated). The caller keeps every buffer alive until the stream has passed the call.
 *     hk_iterate and graphs fork part of an iteration onto a stream the context owns and join it
 *     back, so all of it stays ordered after earlier and before later work on the caller's stream.
 *   - Pointers named "device" must be device memory of the context's GPU; "host" pointers are read
 *     during the call only.
 *   - The library allocates no device memory. The caller allocates the per-set state and the shared
 *     workspace (sizes from hk_state_bytes / hk_workspace_bytes, 256-byte aligned) and owns them.
 *   - Arrays are structure-of-arrays float32: x, y and z (or R, G, B) in three separate arrays.
 *   - Calls on one context are not thread-safe; use one context per host thread.
 */
#ifndef HK_H
#define HK_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HK_VERSION 130

/* status codes */
#define HK_OK 0
#define HK_E_INVALID_ARG (-1)   /* a NULL or out-of-range argument */
#define HK_E_BAD_STATE (-2)     /* call out of order, e.g. hk_iterate before hk_set_kernels */
#define HK_E_SMALL_BUFFER (-3)  /* a caller-allocated buffer is smaller than required */
#define HK_E_HIP (-4)           /* a HIP runtime call failed */
#define HK_E_UNSUPPORTED (-5)   /* a parameter combination this build does not implement */

/* modes */
#define HK_MODE_PPM 0           /* progressive photon mapping: sample = luminance of the photon flux */
#define HK_MODE_VCM 1           /* vertex merging of VCM+: sample = MIS-weighted luminance of the path */

/* test channels (Sec. 5.1 end: luminance by default, one test per RGB channel for chromatic light:
 * the three channels' F are tested against the same critical value and the radius shrinks when any
 * channel rejects; the reported F is the largest channel F) */
#define HK_STATS_LUMA 0
#define HK_STATS_RGB 1

typedef struct hk_ctx hk_ctx;
typedef struct hk_graph hk_graph;

/* Parameters of the estimator (Sec. 5.1 Eq. radiusupdate, Sec. 6 settings). */
typedef struct hk_params {
    float r1;              /* initial radius, > 0 (radii are float32 quantities) */
    float k;               /* shrink ratio in (0, 1), applied as a float32 multiply */
    double alpha_f;        /* significance level of the F-test in (0, 1) */
    double alpha;          /* lower-bound exponent in (0, 1) */
    double rmin;           /* lower-bound scale r_min in [0, r1]; the bound is evaluated in float64 and
                              rounded once to float32 */
    int32_t n_a;           /* annuli; this build supports 2 */
    int32_t n_s;           /* sectors per annulus; this build supports 6 */
    int32_t mode;          /* HK_MODE_PPM or HK_MODE_VCM */
    int32_t stats_channel; /* HK_STATS_LUMA or HK_STATS_RGB */
    float normal_cos_min;  /* a pair counts only if n_kernel . n_photon >= this (when both have normals) */
    int32_t max_iters;     /* iterations a set may run (sizes the critical-value table), 1..65536 */
    float cell_scale;      /* grid cell (y, z) = cell_scale * (radius quantile), x a quarter of it; 0: default */
    float cell_quantile;   /* radius quantile in (0, 1] used for the cell size; 0 selects the default */
    int32_t heavy_cost;    /* kernels whose grid stencil holds more photons are heavy; 0: default */
    int32_t lanes_light;   /* lanes of a wavefront per light kernel: 4, 8 or 16; 0: default */
    int32_t lanes_heavy;   /* lanes of a wavefront per heavy kernel: 16 or 64; 0: default */
    int32_t reserved[5];
} hk_params;

/* One iteration's light vertices of one set. */
typedef struct hk_photons {
    uint64_t J_emitted;    /* light sub-paths traced, stored or not (>= n_stored, >= 1) */
    int64_t n_stored;      /* light vertices in the arrays, >= 0 */
    const float *pos[3];   /* device, n_stored each */
    const float *nrm[3];   /* device or all NULL (no normal test) */
    const float *flux[3];  /* device; PPM: photon flux; VCM: light-vertex throughput */
    const float *mis[3];   /* device, VCM only: light partials dVCM, dVC, dVM (dVC unused) */
} hk_photons;

/* Fills *p with the defaults of the paper's settings: k = 0.7, alpha_F = 0.05, alpha = 0.75,
 * r_min = 0.001 r1, 2 x 6 groups, PPM, luminance test, normal threshold 0.5, 4096 iterations. */
int hk_default_params(double r1, hk_params *p);

/* Creates a context bound to the current HIP device. Validates p (HK_E_INVALID_ARG,
 * HK_E_UNSUPPORTED for n_a != 2 or n_s != 6). *out receives the handle. */
int hk_create(const hk_params *p, hk_ctx **out);
int hk_destroy(hk_ctx *ctx);

/* The context's parameters, with the defaults filled in and any tuning applied. */
int hk_get_params(hk_ctx *ctx, hk_params *out);

/* Changes the performance parameters (cell_scale, heavy_cost, lanes_light, lanes_heavy; 0 selects
 * the default; validated as in hk_create). They change the order of summation, not the estimator:
 * results agree with any other setting to rounding. Applies to later hk_iterate calls and graphs. */
int hk_set_tuning(hk_ctx *ctx, float cell_scale, int heavy_cost, int lanes_light, int lanes_heavy);

/* Bytes of the per-set state for n_kernels hit points, 1 <= n_kernels <= 2^26 - 1 (the caller
 * allocates it on the device). */
int hk_state_bytes(hk_ctx *ctx, int64_t n_kernels, size_t *out);

/* Bytes of the workspace of one hk_iterate call over n_sets sets with n_photons[s] stored light
 * vertices and n_kernels[s] kernels (host arrays). The result also covers any subset of the sets,
 * so one workspace serves every call whose sets are a subset of these, with at most as many
 * photons each. */
int hk_workspace_bytes_batch(hk_ctx *ctx, int n_sets, const int64_t *n_photons, const int64_t *n_kernels,
                             size_t *out);

/* hk_workspace_bytes_batch for one set. */
int hk_workspace_bytes(hk_ctx *ctx, int64_t max_photons, int64_t max_kernels, size_t *out);

/* Initialises set `set_id` (0..255): copies the n hit points into `state` (device, state_bytes(n)),
 * orders them along a Morton curve, computes tangent frames and clears all statistics (t = 0,
 * sums 0, estimate 0, r = r_init or r1). The set's radius scale: r1 (initial radius; <= 0 takes the
 * context's) and rmin (lower-bound scale of Eq. radiusupdate, in [0, r1]; < 0 keeps the context's
 * ratio rmin / r1), so sets of different scales can share a context and a batch. Inputs (device):
 * pos[3]; nrm[3] or NULL (+z); r_init or NULL; VCM only: cam_beta[3] camera throughput, cam_mis[3]
 * partials dVCM, dVC, dVM. `workspace` (device, at least hk_workspace_bytes(ctx, 0, n) bytes, given
 * in workspace_bytes) is scratch for the ordering. Resets the set's iteration count.
 * r_init (device, n radii in the caller's order) must hold finite radii >= the first lower bound
 * r_min (float32): the lower bounds decrease, so every radius then stays at or above the bound and a
 * shrink (Eq. radiusupdate) never makes it grow. With r_init given the call checks it on the device
 * and synchronises `stream`; HK_E_INVALID_ARG (the set stays uninitialised) names how many radii
 * failed. Without r_init it does not synchronise. */
int hk_set_kernels(hk_ctx *ctx, int set_id, int64_t n, double r1, double rmin, const float *const pos[3],
                   const float *const nrm[3], const float *r_init, const float *const cam_beta[3],
                   const float *const cam_mis[3], void *state, void *workspace, size_t workspace_bytes,
                   hipStream_t stream);

/* Runs one iteration (steps 1-6 above) for each of the n_sets (1..256, distinct) sets; ph[s] holds
 * set s's light vertices, state[s] its state, set_ids[s] its id. Each set's grid is built by its own
 * launches; the gather, test and update of up to 64 sets (at most 2^27 - 65 stored light vertices in
 * total, 89,478,421 with the normal test or vertex merging, whose payload records are 48 bytes)
 * run as one launch over a work list spanning those sets, so many small, uneven sets fill the GPU
 * together; a batch of several sets may be gathered in two such launches (phases), the second
 * phase's grids being built while the first phase gathers (hk_gather_phases tells which sets go
 * where). Sets with and without the normal test go to separate launches. The grids are built on
 * streams of the library's own, forked from and joined back to `stream` with events. `workspace` (device,
 * workspace_bytes long) must hold hk_workspace_bytes_batch over the sets (HK_E_SMALL_BUFFER
 * otherwise); a set holds at most 2^27 - 65 stored light vertices per iteration, 89,478,421 with the
 * normal test or vertex merging (HK_E_UNSUPPORTED).
 * Arguments of all sets are checked before any work is enqueued. Non-finite photon values are not
 * rejected: a NaN position never lands in a disk, a NaN flux makes that kernel's F NaN, which keeps
 * the radius (IEEE comparison). */
int hk_iterate(hk_ctx *ctx, int n_sets, const int *set_ids, const hk_photons *ph, void *const *state,
               void *workspace, size_t workspace_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): hk_iterate without a workspace argument. Its scratch is a static
 * array of HK_STATIC_SCRATCH_BYTES in the library's device code, one copy per GPU the library runs
 * on, held from the first hk_create on that GPU until the process ends. The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine) and never profiles. A call whose sets need
 * more scratch than that (hk_workspace_bytes_batch of the sets: about 80 bytes per stored light
 * vertex and 24 per hit point, e.g. up to about 800k light vertices in one call) returns
 * HK_E_SMALL_BUFFER before any work is enqueued; other arguments and errors as hk_iterate. Every
 * call on one GPU shares that GPU's array (it keeps the last call's contents; nothing in it has to
 * start at zero): calls that overlap on one GPU, from any context or stream, race and must be
 * ordered by the caller. */
#define HK_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int hk_iterate_static(hk_ctx *ctx, int n_sets, const int *set_ids, const hk_photons *ph, void *const *state,
                      hipStream_t stream);

/* Captures the launches of one hk_iterate call (same arguments) into a HIP graph, *out. Nothing runs
 * at capture and no set advances. Each hk_graph_launch then runs one iteration of those sets on
 * `stream` (the iteration index, J and the radius bounds come from the device-resident state). The
 * graph reads the photon arrays given here: refill them before each launch; J_emitted and n_stored
 * stay those of the capture. hk_graph_launch fails with HK_E_BAD_STATE if a set was re-initialised
 * since, reached max_iters, or ran with another J in between (capture again). */
int hk_graph_create(hk_ctx *ctx, int n_sets, const int *set_ids, const hk_photons *ph, void *const *state,
                    void *workspace, size_t workspace_bytes, hk_graph **out);
int hk_graph_launch(hk_graph *g, hipStream_t stream);
int hk_graph_destroy(hk_graph *g);

/* ---- light-vertex generation for the box scene (the light pass before the estimator, Sec. 4) ----
 * Scene: the unit box [0,1]^3 without its z = 1 wall, an isotropic point light strictly inside it
 * and an opaque sphere. Light sub-path j of iteration i of set s draws Philox4x32-10 blocks (Salmon
 * et al., SC 2011) with counter (j, i, s, b) and key (seed mod 2^32, seed div 2^32), b = 0..7; a word
 * x gives u = (x >> 8) 2^-24. Block b holds the direction attempts 2b (words 0, 1) and 2b + 1 (words
 * 2, 3): a = 2u - 1, c = 2u' - 1, q = a a + c c, the first attempt with 0 < q < 1 gives the unit
 * direction (a f, c f, 1 - 2q), f = 2 sqrt(1 - q) (Marsaglia 1972). The vertex is the first wall hit
 * (per-axis exit distances, the smallest on the first of x, y, z that attains it); the sub-path
 * leaves no vertex when it escapes through the open top, when the sphere's near intersection lies
 * in (0, t), or when all 16 attempts fail. Every float32 operation is one correctly rounded IEEE
 * operation, in the order stated, so the output is bit-reproducible by any implementation of this
 * definition. */
typedef struct hk_box_scene {
    float light[3];        /* point light, each coordinate in (0, 1) */
    float sphere_c[3];     /* occluder centre (finite) */
    float sphere_r;        /* occluder radius, >= 0 (0: no occluder) */
    float power;           /* flux per channel carried by every vertex, e.g. 4 pi I for intensity I */
} hk_box_scene;

/* Writes the J slots of set `set_id`'s next iteration (its index is read on the device from `state`,
 * the set's hk_set_kernels state) into pos, nrm and flux (device, J floats each, structure of arrays).
 * A slot with a vertex holds its position (the hit coordinate exactly 0 or 1), the wall's inward unit
 * normal and `power` in R, G and B; a slot without one holds NaN positions, a zero normal and zero
 * flux, which the estimator never gathers. When mis is non-NULL (all three device arrays, or NULL),
 * it receives the vertex-merging partials of each vertex: dVCM = (4 pi t^2) / |d_a| in float32
 * (t the distance from the light, d_a the unit direction's component on the hit axis: the reciprocal
 * of the area density with which the light pass reaches the vertex), dVC = dVM = 0; zero in empty
 * slots. The batch for hk_iterate is then {J_emitted = J, n_stored = J, pos, nrm, flux[, mis]}.
 * J in [0, 2^27 - 1]. Asynchronous on `stream`; nothing advances. */
int hk_emit_box(hk_ctx *ctx, int set_id, const void *state, const hk_box_scene *scene, uint64_t seed,
                int64_t J, float *const pos[3], float *const nrm[3], float *const flux[3], float *const mis[3],
                hipStream_t stream);

/* Vertex connection for the box scene (the VC sum of Eq. VCM-estimator, here the connection of each
 * camera vertex x to the point light): adds w_VC beta_C I cos(theta_x) V(x) / d^2 per channel to the
 * set's running estimate for the iteration about to run, with the balance-heuristic weight of Eq.
 * mis-weight against merging, w_VC = 1 / (1 + J pi r^2 cos(theta_x) / (4 pi d^2)), r the camera
 * vertex's current radius (the one the next hk_iterate merges with), J = J_emitted of that
 * iteration, I = power / (4 pi), V the float32 shadow test of the segment x -> light against the
 * sphere (with w = light - x, dist = sqrt((w_x w_x + w_y w_y) + w_z w_z), u = w / dist, o = x - C,
 * B = (u_x o_x + u_y o_y) + u_z o_z, Q = ((o_x o_x + o_y o_y) + o_z o_z) - R R: blocked when
 * B B - Q > 0 and -B - sqrt(B B - Q) lies in (0, dist)). Merging then carries the complementary
 * weight when the light vertices carry hk_emit_box's partials and the camera partials are zero.
 * Needs vertex-merging mode and camera vertices with normals (HK_E_BAD_STATE otherwise). Call it on
 * the same stream before the hk_iterate of the iteration. */
int hk_connect_box(hk_ctx *ctx, int set_id, void *state, const hk_box_scene *scene, uint64_t J_emitted,
                   hipStream_t stream);

/* hk_graph_create with the generation of every set's batch in front: each launch of the graph
 * writes the batches ph[s] (device arrays; they must be writable, with n_stored == J_emitted, the
 * normal arrays given, and in vertex-merging mode the mis arrays) with hk_emit_box's definition for
 * scenes[s] and seeds[s] and the set's current iteration, then (flags & HK_BOX_CONNECT) runs
 * hk_connect_box for every set, then the iteration. One replay is one complete iteration with no
 * host work beyond the launch. */
#define HK_BOX_CONNECT 1
int hk_graph_create_box(hk_ctx *ctx, int n_sets, const int *set_ids, const hk_box_scene *scenes,
                        const uint64_t *seeds, const hk_photons *ph, void *const *state, void *workspace,
                        size_t workspace_bytes, int flags, hk_graph **out);

/* Times one iteration of the given sets for each of 48 settings (cell_scale 0.35 / 0.5 / 0.7 / 1 x
 * lanes_light 4 / 8 / 16 x heavy_cost 1024 / 2048 / 4096 / 16384; the fastest of three runs of each)
 * and keeps the fastest setting in the context
 * (copied to *chosen when non-NULL). Each trial runs on scratch[s] (device, hk_state_bytes of the
 * set, distinct from state[s]) after copying state[s] into it, so the states and the sets'
 * iteration counts are left unchanged. Synchronises `stream`. */
int hk_autotune(hk_ctx *ctx, int n_sets, const int *set_ids, const hk_photons *ph, void *const *state,
                void *const *scratch, void *workspace, size_t workspace_bytes, hipStream_t stream,
                hk_params *chosen);

/* ---- learned radius proposal (an addition to the paper's method; the F-test keeps judging) ------
 * Features of a hit point: the light vertices of one batch in 8 equi-areal rings (ring b holds
 * b/8 <= d^2/R^2 < (b+1)/8) at the four radii R = r1, r1/2, r1/4, r1/8, with the gather's inside-disk
 * and normal tests; encoded as log1p(count) / 8, then the hit point's normal (3) and an iteration
 * code (1): 36 bfloat16 values per hit point (uint16 bit patterns, row-major n x 36). Network: 36 ->
 * 64 -> 64 -> 1 with ReLU, weights in bfloat16 on the matrix cores, float32 biases and accumulation,
 * trained for the mean squared error by Adam (beta1 0.9, beta2 0.999, eps 1e-8) on float32 master
 * parameters. Parameter vector (float32, hk_mlp_param_count() = 6593 values): W1 (36 x 64, row =
 * input), b1 (64), W2 (64 x 64, row = input), b2 (64), w3 (64), b3. The network state (device,
 * hk_mlp_state_bytes, 256-byte aligned) is owned by the caller. */
int hk_mlp_param_count(void);
int hk_mlp_state_bytes(size_t *out);

/* Device workspace of hk_mlp_grad / hk_mlp_train_step for n samples. */
int hk_mlp_workspace_bytes(int64_t n, size_t *out);

/* Loads parameters (device float32 array of hk_mlp_param_count values) and clears Adam's moments
 * and step count. */
int hk_mlp_set_params(hk_ctx *ctx, void *mlp, const float *theta, hipStream_t stream);

/* Copies the float32 master parameters to theta_out (device). */
int hk_mlp_get_params(hk_ctx *ctx, const void *mlp, float *theta_out, hipStream_t stream);

/* y[i] = network(feat[i]) for n samples (device arrays). */
int hk_mlp_forward(hk_ctx *ctx, const void *mlp, const uint16_t *feat, int64_t n, float *y, hipStream_t stream);

/* Gradient of the mean squared error (1/n) sum (y_i - label_i)^2 over the n samples, written to
 * grad_out (device, hk_mlp_param_count() + 1 floats: the gradient, then the sum of squared errors);
 * no update. workspace: hk_mlp_workspace_bytes(n). */
int hk_mlp_grad(hk_ctx *ctx, const void *mlp, const uint16_t *feat, const float *label, int64_t n, float *grad_out,
                void *workspace, size_t workspace_bytes, hipStream_t stream);

/* One Adam step on the mean squared error of the n samples (one mini-batch) with learning rate lr. */
int hk_mlp_train_step(hk_ctx *ctx, void *mlp, const uint16_t *feat, const float *label, int64_t n, float lr,
                      void *workspace, size_t workspace_bytes, hipStream_t stream);

/* Features of set set_id's hit points from one batch of light vertices *ph (sorted into a grid of
 * cell r1 in the workspace, hk_workspace_bytes(ctx, n_stored, H)); it_code is the last input of
 * every row. feat (device, H x 36 bfloat16) and counts (device, H x 32 uint32, or NULL) are in the
 * caller's original hit-point order. The set's iteration state is not changed. */
int hk_mlp_features(hk_ctx *ctx, int set_id, void *state, const hk_photons *ph, float it_code, uint16_t *feat,
                    uint32_t *counts, void *workspace, size_t workspace_bytes, hipStream_t stream);

/* Proposal for the set's next iteration i + 1 from network outputs y (device, H floats, original
 * order, predicting log(r / r1)): r <- min(max(r1 exp(y + margin), lb_{i+1}), r) in float32, so a
 * radius never grows and never drops below the bound of Eq. radiusupdate; margin > 0 proposes
 * larger radii than predicted (the F-test can still shrink them, never grow them). Hit points whose
 * radius changes start their retained statistics afresh (t = 0, sums 0); the estimate so far is
 * kept. */
int hk_mlp_propose(hk_ctx *ctx, int set_id, void *state, const float *y, float margin, hipStream_t stream);

/* Radiance estimate L = f_r tau / N per channel (f_r = 1/pi), in the caller's original kernel order.
 * out_rgb[3]: device arrays of n floats. */
int hk_read_radiance(hk_ctx *ctx, int set_id, const void *state, float *const out_rgb[3], hipStream_t stream);

/* Current radii (device float[n]), original order. */
int hk_read_radii(hk_ctx *ctx, int set_id, const void *state, float *out, hipStream_t stream);

/* Last iteration's per-kernel values, original order (any pointer may be NULL): in-disk count,
 * F (NaN when undefined), critical value used, shrink decision (1 = shrunk), kept iterations t. */
int hk_read_debug(hk_ctx *ctx, int set_id, const void *state, uint32_t *count, double *F, double *Fc,
                  uint8_t *decision, uint32_t *t, hipStream_t stream);

/* Retained group sums in float64 (device, row-major, original order): S and Q, n x 12 each with the
 * luminance test and n x 36 with one test per channel (column = channel * 12 + group), as the state
 * holds them, and the estimate tau (n x 3, a float32 value plus its collected rounding error). */
int hk_read_sums(hk_ctx *ctx, int set_id, const void *state, double *S, double *Q, double *tau,
                 hipStream_t stream);

/* Running totals of the set since hk_set_kernels, written to out (device, 4 x uint64): [0]
 * iterations, [1] in-disk (kernel, photon) pairs, [2] kernel x photon candidate tests, [3] grid cells
 * of the last iteration. */
int hk_read_stats(hk_ctx *ctx, int set_id, const void *state, uint64_t *out, hipStream_t stream);

/* Host routine: (1 - alpha) quantile of the F(d1, d2) distribution in float64, the same routine the
 * device evaluates for the critical value (Sec. 3.2.2). Returns NaN for invalid arguments. */
double hk_f_quantile(double d1, double d2, double alpha);

/* Timing of the hk_iterate calls since enabling (hipEvents on the caller's stream; graphs are not
 * timed): hk_profile_enable(ctx, 1) starts recording, hk_profile_read(ctx, out, n) synchronises on
 * the last event and writes up to n values: phase totals in milliseconds [0] iteration plans and
 * grid builds (of a batch's second gather phase, the part not hidden behind the first gather),
 * [1] wait for the critical values beyond the grid builds (they run on a second stream beside them),
 * [2] work lists and set table, [3] the gather / test / update launches alone, [4] radius histogram
 * and pair tally; then [5] the number of gather launches timed (two per batch of two or more sets:
 * the second phase's grids are built while the first phase's gather runs); then [6], [7] the
 * gather launches' milliseconds of first and of second phases, [8], [9] their numbers. */
int hk_profile_enable(hk_ctx *ctx, int on);
int hk_profile_read(hk_ctx *ctx, double *out, int n);

/* Which gather phase (0: first, 1: second) each of the n_sets sets would take in an hk_iterate call
 * with the same set_ids and light vertices: phase[s] for set_ids[s]. ph[s].n_stored is read, and
 * whether ph[s].nrm[0] is NULL; no pointer is dereferenced. Host-side, nothing is enqueued. Sets
 * must have kernels (HK_E_BAD_STATE); bad arguments (ids out of range or repeated, NULL arrays)
 * give HK_E_INVALID_ARG. Used to attribute work
 * to the two gather launches of a batch when timing them. */
int hk_gather_phases(hk_ctx *ctx, int n_sets, const int *set_ids, const hk_photons *ph, int *phase);

int hk_version(void);
const char *hk_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HK_H */

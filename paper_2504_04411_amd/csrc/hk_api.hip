// C ABI of libhk (declared in include/hk.h): argument checking, state / workspace carve-up and the
// per-iteration launch sequence. All device work is enqueued on the caller's stream; the library
// owns no device memory.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "hk_internal.h"
#include "hk_kernels.h"

using namespace hk;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) return fail(HK_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int MAX_SETS = 256;

struct SetInfo {
    bool init = false;
    int64_t H = 0;
    int iter = 0;              // completed iterations
    bool has_nrm = false;
    bool J_const = true;       // every J so far equal -> table entries t < iter stay valid
    uint64_t J_first = 0;
    int fc_valid_upto = 0;     // fctab[1..fc_valid_upto] computed for the current J history
};

struct ProfEv {
    hipEvent_t e[4];
};

}  // namespace

struct hk_ctx {
    hk_params p;
    int device = 0;
    SetInfo sets[MAX_SETS];
    bool prof = false;
    std::vector<ProfEv> ev_used, ev_free;
    double prof_ms[4] = {0, 0, 0, 0};
};

static bool finite_pos(float x) { return isfinite(x) && x > 0.0f; }

extern "C" int hk_version(void) { return HK_VERSION; }

extern "C" const char *hk_last_error(void) { return g_err.c_str(); }

extern "C" int hk_default_params(double r1, hk_params *p)
{
    if (!p) return fail(HK_E_INVALID_ARG, "hk_default_params: p is NULL");
    memset(p, 0, sizeof *p);
    p->r1 = (float)r1;
    p->k = 0.7f;
    p->alpha_f = 0.05;
    p->alpha = 0.75;
    p->rmin = 0.001 * r1;
    p->n_a = 2;
    p->n_s = 6;
    p->mode = HK_MODE_PPM;
    p->stats_channel = HK_STATS_LUMA;
    p->normal_cos_min = 0.5f;
    p->max_iters = 4096;
    p->cell_scale = 1.0f;
    p->cell_quantile = 0.5f;
    p->heavy_cost = 4096;
    p->lanes_light = 8;
    p->lanes_heavy = 64;
    return HK_OK;
}

extern "C" int hk_create(const hk_params *p, hk_ctx **out)
{
    if (!p || !out) return fail(HK_E_INVALID_ARG, "hk_create: NULL argument");
    *out = nullptr;
    if (!finite_pos(p->r1)) return fail(HK_E_INVALID_ARG, "r1 must be finite and > 0");
    if (!(p->k > 0.0f && p->k < 1.0f)) return fail(HK_E_INVALID_ARG, "k must be in (0, 1)");
    if (!(p->alpha_f > 0.0 && p->alpha_f < 1.0)) return fail(HK_E_INVALID_ARG, "alpha_f must be in (0, 1)");
    if (!(p->alpha > 0.0 && p->alpha < 1.0)) return fail(HK_E_INVALID_ARG, "alpha must be in (0, 1)");
    if (!(p->rmin >= 0.0 && p->rmin <= (double)p->r1 * (1.0 + 1e-7)))
        return fail(HK_E_INVALID_ARG, "rmin must be in [0, r1]");
    if (p->n_a != 2 || p->n_s != 6) return fail(HK_E_UNSUPPORTED, "only n_a = 2, n_s = 6 is implemented");
    if (p->mode != HK_MODE_PPM && p->mode != HK_MODE_VCM) return fail(HK_E_INVALID_ARG, "unknown mode");
    if (p->stats_channel != HK_STATS_LUMA) return fail(HK_E_UNSUPPORTED, "only the luminance test is implemented");
    if (!(p->normal_cos_min >= -1.0f && p->normal_cos_min <= 1.0f))
        return fail(HK_E_INVALID_ARG, "normal_cos_min must be in [-1, 1]");
    if (p->max_iters < 1 || p->max_iters > 65536) return fail(HK_E_INVALID_ARG, "max_iters must be in [1, 65536]");
    if (!(p->cell_scale >= 0.0f && isfinite(p->cell_scale))) return fail(HK_E_INVALID_ARG, "bad cell_scale");
    if (!(p->cell_quantile >= 0.0f && p->cell_quantile <= 1.0f)) return fail(HK_E_INVALID_ARG, "bad cell_quantile");
    if (p->lanes_light != 0 && p->lanes_light != 4 && p->lanes_light != 8 && p->lanes_light != 16)
        return fail(HK_E_INVALID_ARG, "lanes_light must be 4, 8 or 16");
    if (p->lanes_heavy != 0 && p->lanes_heavy != 16 && p->lanes_heavy != 64)
        return fail(HK_E_INVALID_ARG, "lanes_heavy must be 16 or 64");
    hk_ctx *c = new (std::nothrow) hk_ctx();
    if (!c) return fail(HK_E_INVALID_ARG, "out of host memory");
    c->p = *p;
    if (c->p.cell_scale == 0.0f) c->p.cell_scale = 1.0f;
    if (c->p.cell_quantile == 0.0f) c->p.cell_quantile = 0.5f;
    if (c->p.heavy_cost <= 0) c->p.heavy_cost = 4096;
    if (c->p.lanes_light == 0) c->p.lanes_light = 8;
    if (c->p.lanes_heavy == 0) c->p.lanes_heavy = 64;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(HK_E_HIP, "hipGetDevice failed");
    }
    *out = c;
    return HK_OK;
}

extern "C" int hk_destroy(hk_ctx *ctx)
{
    if (!ctx) return fail(HK_E_INVALID_ARG, "hk_destroy: NULL context");
    for (auto &v : {&ctx->ev_used, &ctx->ev_free})
        for (auto &pe : *v)
            for (auto e : pe.e) (void)hipEventDestroy(e);
    delete ctx;
    return HK_OK;
}

static Layout layout_of(const hk_ctx *ctx, int64_t H) { return make_layout(H, ctx->p.max_iters, false); }

extern "C" int hk_state_bytes(hk_ctx *ctx, int64_t n_kernels, size_t *out)
{
    if (!ctx || !out) return fail(HK_E_INVALID_ARG, "hk_state_bytes: NULL argument");
    if (n_kernels < 1 || n_kernels > (int64_t)INT32_MAX - 64) return fail(HK_E_INVALID_ARG, "n_kernels out of range");
    *out = layout_of(ctx, n_kernels).total;
    return HK_OK;
}

extern "C" int hk_workspace_bytes(hk_ctx *ctx, int64_t max_photons, int64_t max_kernels, size_t *out)
{
    if (!ctx || !out) return fail(HK_E_INVALID_ARG, "hk_workspace_bytes: NULL argument");
    if (max_photons < 0 || max_photons > (int64_t)UINT32_MAX - 1024 || max_kernels < 0 ||
        max_kernels > (int64_t)INT32_MAX - 64)
        return fail(HK_E_INVALID_ARG, "sizes out of range");
    *out = make_ws_layout(max_photons, max_kernels).total;
    return HK_OK;
}

static bool aligned(const void *p) { return ((uintptr_t)p & 255u) == 0; }

extern "C" int hk_set_kernels(hk_ctx *ctx, int set_id, int64_t n, const float *const pos[3], const float *const nrm[3],
                              const float *r_init, const float *const cam_beta[3], const float *const cam_mis[3],
                              void *state, void *workspace, size_t workspace_bytes, hipStream_t stream)
{
    if (!ctx) return fail(HK_E_INVALID_ARG, "hk_set_kernels: NULL context");
    if (set_id < 0 || set_id >= MAX_SETS) return fail(HK_E_INVALID_ARG, "set_id out of range");
    if (n < 1 || n > (int64_t)INT32_MAX - 64) return fail(HK_E_INVALID_ARG, "n out of range");
    if (!pos || !pos[0] || !pos[1] || !pos[2]) return fail(HK_E_INVALID_ARG, "pos is NULL");
    if (!state || !aligned(state)) return fail(HK_E_INVALID_ARG, "state must be non-NULL and 256-byte aligned");
    if (!workspace || !aligned(workspace)) return fail(HK_E_INVALID_ARG, "workspace must be 256-byte aligned");
    const bool vcm = ctx->p.mode == HK_MODE_VCM;
    const bool has_nrm = nrm && nrm[0];
    if (has_nrm && (!nrm[1] || !nrm[2])) return fail(HK_E_INVALID_ARG, "nrm must be all NULL or all set");
    if (vcm && (!cam_beta || !cam_beta[0] || !cam_beta[1] || !cam_beta[2] || !cam_mis || !cam_mis[0] ||
                !cam_mis[2]))
        return fail(HK_E_INVALID_ARG, "vertex merging needs cam_beta[3] and cam_mis (dVCM, -, dVM)");
    const WsLayout W = make_ws_layout(0, n);
    if (workspace_bytes < W.total)
        return fail(HK_E_SMALL_BUFFER, "workspace of %zu bytes, %zu needed", workspace_bytes, W.total);
    HIP_TRY(hipSetDevice(ctx->device));
    const Layout L = layout_of(ctx, n);
    char *w = static_cast<char *>(workspace);
    InitLaunch g{};
    g.st = make_view(state, L);
    for (int a = 0; a < 3; ++a) {
        g.src.pos[a] = pos[a];
        g.src.nrm[a] = has_nrm ? nrm[a] : nullptr;
        g.src.cam_beta[a] = vcm ? cam_beta[a] : nullptr;
        g.src.cam_mis[a] = vcm ? cam_mis[a] : nullptr;
    }
    g.src.r_init = r_init;
    g.n = n;
    g.max_iters = ctx->p.max_iters;
    g.r1 = ctx->p.r1;
    g.vcm = vcm;
    g.nsq = NSQ;
    g.keyA = reinterpret_cast<uint32_t *>(w + W.keyA);
    g.keyB = reinterpret_cast<uint32_t *>(w + W.keyB);
    g.valA = reinterpret_cast<uint32_t *>(w + W.valA);
    g.valB = reinterpret_cast<uint32_t *>(w + W.valB);
    g.hist = reinterpret_cast<uint32_t *>(w + W.hist);
    g.part = reinterpret_cast<uint32_t *>(w + W.part);
    init_set(g, stream);
    HIP_TRY(hipGetLastError());
    SetInfo &S = ctx->sets[set_id];
    S = SetInfo();
    S.init = true;
    S.H = n;
    S.has_nrm = has_nrm;
    return HK_OK;
}

static ProfEv *prof_slot(hk_ctx *ctx)
{
    if (ctx->ev_free.empty()) {
        ProfEv pe;
        for (auto &e : pe.e)
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
        ctx->ev_free.push_back(pe);
    }
    ctx->ev_used.push_back(ctx->ev_free.back());
    ctx->ev_free.pop_back();
    return &ctx->ev_used.back();
}

extern "C" int hk_iterate(hk_ctx *ctx, int n_sets, const int *set_ids, const hk_photons *ph, void *const *state,
                          void *workspace, size_t workspace_bytes, hipStream_t stream)
{
    if (!ctx) return fail(HK_E_INVALID_ARG, "hk_iterate: NULL context");
    if (n_sets < 1 || !set_ids || !ph || !state) return fail(HK_E_INVALID_ARG, "hk_iterate: bad set arguments");
    if (!workspace || !aligned(workspace)) return fail(HK_E_INVALID_ARG, "workspace must be 256-byte aligned");
    const bool vcm = ctx->p.mode == HK_MODE_VCM;
    // validate everything before enqueuing anything
    for (int s = 0; s < n_sets; ++s) {
        const int id = set_ids[s];
        if (id < 0 || id >= MAX_SETS) return fail(HK_E_INVALID_ARG, "set id %d out of range", id);
        if (!ctx->sets[id].init) return fail(HK_E_BAD_STATE, "set %d has no kernels (call hk_set_kernels)", id);
        if (ctx->sets[id].iter >= ctx->p.max_iters) return fail(HK_E_BAD_STATE, "set %d reached max_iters", id);
        if (!state[s] || !aligned(state[s])) return fail(HK_E_INVALID_ARG, "state of set %d not aligned", id);
        const hk_photons &P = ph[s];
        if (P.J_emitted < 1 || P.n_stored < 0 || (uint64_t)P.n_stored > P.J_emitted)
            return fail(HK_E_INVALID_ARG, "set %d: need 1 <= J_emitted and 0 <= n_stored <= J_emitted", id);
        if (P.J_emitted > (uint64_t)1 << 52) return fail(HK_E_INVALID_ARG, "J_emitted too large");
        if (P.n_stored >= ((int64_t)1 << 27))
            return fail(HK_E_UNSUPPORTED, "set %d: at most 2^27 - 1 stored light vertices per set", id);
        if (P.n_stored > 0) {
            for (int a = 0; a < 3; ++a)
                if (!P.pos[a] || !P.flux[a]) return fail(HK_E_INVALID_ARG, "set %d: pos/flux is NULL", id);
            if (vcm && (!P.mis[0] || !P.mis[2])) return fail(HK_E_INVALID_ARG, "set %d: mis partials needed", id);
            if (ctx->sets[id].has_nrm && !P.nrm[0] && (P.nrm[1] || P.nrm[2]))
                return fail(HK_E_INVALID_ARG, "set %d: nrm must be all NULL or all set", id);
        }
        const WsLayout W = make_ws_layout(P.n_stored, ctx->sets[id].H);
        if (workspace_bytes < W.total)
            return fail(HK_E_SMALL_BUFFER, "workspace of %zu bytes, %zu needed", workspace_bytes, W.total);
    }
    HIP_TRY(hipSetDevice(ctx->device));
    const hk_params &p = ctx->p;
    for (int s = 0; s < n_sets; ++s) {
        const int id = set_ids[s];
        SetInfo &S = ctx->sets[id];
        const hk_photons &P = ph[s];
        const Layout L = layout_of(ctx, S.H);
        const StateView st = make_view(state[s], L);
        const WsLayout W = make_ws_layout(P.n_stored, S.H);
        char *w = static_cast<char *>(workspace);
        const int i = S.iter + 1;
        if (i == 1) S.J_first = P.J_emitted;
        if (P.J_emitted != S.J_first) S.J_const = false;
        ProfEv *pe = ctx->prof ? prof_slot(ctx) : nullptr;
        if (ctx->prof && !pe) return fail(HK_E_HIP, "hipEventCreate failed");
        if (pe) HIP_TRY(hipEventRecord(pe->e[0], stream));

        launch_plan(st.hdr, st.mprefix, i, (double)P.J_emitted, p.cell_scale, p.cell_quantile, W.max_cells, stream);
        GridLaunch g{};
        g.hdr = st.hdr;
        for (int a = 0; a < 3; ++a) {
            g.src.pos[a] = P.pos[a];
            g.src.nrm[a] = S.has_nrm ? P.nrm[a] : nullptr;
            g.src.flux[a] = P.flux[a];
            g.src.mis[a] = vcm ? P.mis[a] : nullptr;
        }
        const bool nrm_test = S.has_nrm && P.nrm[0] != nullptr;
        if (!nrm_test)
            for (int a = 0; a < 3; ++a) g.src.nrm[a] = nullptr;
        g.n = P.n_stored;
        g.keyA = reinterpret_cast<uint32_t *>(w + W.keyA);
        g.keyB = reinterpret_cast<uint32_t *>(w + W.keyB);
        g.valA = reinterpret_cast<uint32_t *>(w + W.valA);
        g.valB = reinterpret_cast<uint32_t *>(w + W.valB);
        g.hist = reinterpret_cast<uint32_t *>(w + W.hist);
        g.part = reinterpret_cast<uint32_t *>(w + W.part);
        g.part3 = reinterpret_cast<uint32_t *>(w + W.part3);
        g.cstart = reinterpret_cast<uint32_t *>(w + W.cstart);
        g.pay = reinterpret_cast<float4 *>(w + W.pay);
        g.pstride = P.n_stored;
        g.ncells_bound = W.max_cells;
        build_grid(g, stream);
        if (pe) HIP_TRY(hipEventRecord(pe->e[1], stream));

        // critical values for t = 1..i; with a constant J only the new entry t = i changes
        const int t_lo = (S.J_const && S.fc_valid_upto == i - 1) ? i : 1;
        launch_fcrit(st.fctab, st.mprefix, i, t_lo, i, p.alpha_f, stream);
        S.fc_valid_upto = S.J_const ? i : 0;
        if (pe) HIP_TRY(hipEventRecord(pe->e[2], stream));

        ListLaunch wl{};
        wl.H = S.H;
        wl.hdr = st.hdr;
        wl.cstart = g.cstart;
        for (int k = 0; k < 3; ++k) wl.kp[k] = st.pos[k];
        wl.r = st.r;
        wl.heavy_cost = (uint32_t)p.heavy_cost;
        wl.flag = reinterpret_cast<uint32_t *>(w + W.flag);
        wl.offs = reinterpret_cast<uint32_t *>(w + W.offs);
        wl.part2 = reinterpret_cast<uint32_t *>(w + W.part2);
        wl.heavy = reinterpret_cast<uint32_t *>(w + W.heavy);
        wl.light = reinterpret_cast<uint32_t *>(w + W.light);
        wl.counts = reinterpret_cast<uint32_t *>(w + W.counts);
        build_work_list(wl, stream);

        GatherArgs a{};
        a.H = S.H;
        a.hdr = st.hdr;
        a.cstart = g.cstart;
        a.payA = g.pay;
        a.payB = g.pay + g.pstride;
        a.payC = g.pay + 2 * g.pstride;
        a.npay = (uint32_t)P.n_stored;
        a.heavy = wl.heavy;
        a.light = wl.light;
        a.counts = wl.counts;
        a.lanes_light = p.lanes_light;
        a.lanes_heavy = p.lanes_heavy;
        for (int k = 0; k < 3; ++k) {
            a.kp[k] = st.pos[k];
            a.kn[k] = st.nrm[k];
            a.ku[k] = st.u[k];
            a.kv[k] = st.v[k];
            a.cb[k] = st.cb[k];
        }
        a.r = st.r;
        a.t = st.t;
        a.nseen = st.nseen;
        a.cnt = st.cnt;
        a.dec = st.dec;
        a.sq0 = st.sq[0];
        a.tau0 = st.tau[0];
        a.astride = (uint32_t)(align256(sizeof(float) * (size_t)S.H) / sizeof(float));
        a.F = st.F;
        a.Fc = st.Fc;
        a.cdvcm = st.cdvcm;
        a.cdvm = st.cdvm;
        a.fctab = st.fctab;
        a.mprefix = st.mprefix;
        a.iter = i;
        a.Jf = (float)P.J_emitted;
        a.lb = (float)(p.rmin * sqrt(pow((double)(i + 1), p.alpha - 1.0)));
        a.k = p.k;
        a.cos_min = p.normal_cos_min;
        a.r1 = p.r1;
        launch_gather(a, nrm_test, vcm, stream);
        if (pe) HIP_TRY(hipEventRecord(pe->e[3], stream));
        HIP_TRY(hipGetLastError());
        S.iter = i;
    }
    return HK_OK;
}

// ------------------------------------------------------------------------------------------------
// reads
// ------------------------------------------------------------------------------------------------

namespace {

__global__ void read_radiance_kernel(StateView st, int64_t n, float scale, float *oR, float *oG, float *oB)
{
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const uint32_t j = st.orig[s];
    oR[j] = (st.tau[0][s] - st.tau[1][s]) * scale;
    oG[j] = (st.tau[2][s] - st.tau[3][s]) * scale;
    oB[j] = (st.tau[4][s] - st.tau[5][s]) * scale;
}

__global__ void read_radii_kernel(StateView st, int64_t n, float *out)
{
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s < n) out[st.orig[s]] = st.r[s];
}

__global__ void read_debug_kernel(StateView st, int64_t n, uint32_t *count, double *F, double *Fc, uint8_t *dec,
                                  uint32_t *t)
{
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const uint32_t j = st.orig[s];
    if (count) count[j] = st.cnt[s];
    if (F) F[j] = st.F[s];
    if (Fc) Fc[j] = st.Fc[s];
    if (dec) dec[j] = (uint8_t)st.dec[s];
    if (t) t[j] = st.t[s];
}

__global__ void read_sums_kernel(StateView st, int64_t n, double *S, double *Q, double *tau)
{
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    const uint32_t j = st.orig[s];
    for (int g = 0; g < NG; ++g) {
        if (S) S[(int64_t)j * NG + g] = (double)st.sq[4 * g][s] - (double)st.sq[4 * g + 1][s];
        if (Q) Q[(int64_t)j * NG + g] = (double)st.sq[4 * g + 2][s] - (double)st.sq[4 * g + 3][s];
    }
    if (tau)
        for (int c = 0; c < 3; ++c) tau[(int64_t)j * 3 + c] = (double)st.tau[2 * c][s] - (double)st.tau[2 * c + 1][s];
}

}  // namespace

static int check_read(hk_ctx *ctx, int set_id, const void *state)
{
    if (!ctx) return fail(HK_E_INVALID_ARG, "NULL context");
    if (set_id < 0 || set_id >= MAX_SETS) return fail(HK_E_INVALID_ARG, "set_id out of range");
    if (!ctx->sets[set_id].init) return fail(HK_E_BAD_STATE, "set %d has no kernels", set_id);
    if (!state || !aligned(state)) return fail(HK_E_INVALID_ARG, "state must be 256-byte aligned");
    return HK_OK;
}

extern "C" int hk_read_radiance(hk_ctx *ctx, int set_id, const void *state, float *const out_rgb[3],
                                hipStream_t stream)
{
    int rc = check_read(ctx, set_id, state);
    if (rc) return rc;
    if (!out_rgb || !out_rgb[0] || !out_rgb[1] || !out_rgb[2]) return fail(HK_E_INVALID_ARG, "out_rgb is NULL");
    const SetInfo &S = ctx->sets[set_id];
    HIP_TRY(hipSetDevice(ctx->device));
    const StateView st = make_view(const_cast<void *>(state), layout_of(ctx, S.H));
    const float scale = INV_PI_F / (float)(S.iter > 0 ? S.iter : 1);
    read_radiance_kernel<<<(int)cdiv(S.H, 256), 256, 0, stream>>>(st, S.H, scale, out_rgb[0], out_rgb[1], out_rgb[2]);
    HIP_TRY(hipGetLastError());
    return HK_OK;
}

extern "C" int hk_read_radii(hk_ctx *ctx, int set_id, const void *state, float *out, hipStream_t stream)
{
    int rc = check_read(ctx, set_id, state);
    if (rc) return rc;
    if (!out) return fail(HK_E_INVALID_ARG, "out is NULL");
    const SetInfo &S = ctx->sets[set_id];
    HIP_TRY(hipSetDevice(ctx->device));
    const StateView st = make_view(const_cast<void *>(state), layout_of(ctx, S.H));
    read_radii_kernel<<<(int)cdiv(S.H, 256), 256, 0, stream>>>(st, S.H, out);
    HIP_TRY(hipGetLastError());
    return HK_OK;
}

extern "C" int hk_read_debug(hk_ctx *ctx, int set_id, const void *state, uint32_t *count, double *F, double *Fc,
                             uint8_t *decision, uint32_t *t, hipStream_t stream)
{
    int rc = check_read(ctx, set_id, state);
    if (rc) return rc;
    const SetInfo &S = ctx->sets[set_id];
    HIP_TRY(hipSetDevice(ctx->device));
    const StateView st = make_view(const_cast<void *>(state), layout_of(ctx, S.H));
    read_debug_kernel<<<(int)cdiv(S.H, 256), 256, 0, stream>>>(st, S.H, count, F, Fc, decision, t);
    HIP_TRY(hipGetLastError());
    return HK_OK;
}

extern "C" int hk_read_sums(hk_ctx *ctx, int set_id, const void *state, double *S_out, double *Q_out,
                            double *tau_out, hipStream_t stream)
{
    int rc = check_read(ctx, set_id, state);
    if (rc) return rc;
    const SetInfo &S = ctx->sets[set_id];
    HIP_TRY(hipSetDevice(ctx->device));
    const StateView st = make_view(const_cast<void *>(state), layout_of(ctx, S.H));
    read_sums_kernel<<<(int)cdiv(S.H, 256), 256, 0, stream>>>(st, S.H, S_out, Q_out, tau_out);
    HIP_TRY(hipGetLastError());
    return HK_OK;
}

namespace {
__global__ void read_stats_kernel(const SetHeader *hdr, uint64_t *out)
{
    if (threadIdx.x == 0) {
        out[0] = hdr->n_launch;
        out[1] = hdr->n_pairs;
        out[2] = hdr->n_cand;
        out[3] = (uint64_t)hdr->ncells;
    }
}
}  // namespace

extern "C" int hk_read_stats(hk_ctx *ctx, int set_id, const void *state, uint64_t *out, hipStream_t stream)
{
    int rc = check_read(ctx, set_id, state);
    if (rc) return rc;
    if (!out) return fail(HK_E_INVALID_ARG, "out is NULL");
    const SetInfo &S = ctx->sets[set_id];
    HIP_TRY(hipSetDevice(ctx->device));
    const StateView st = make_view(const_cast<void *>(state), layout_of(ctx, S.H));
    read_stats_kernel<<<1, 64, 0, stream>>>(st.hdr, out);
    HIP_TRY(hipGetLastError());
    return HK_OK;
}

extern "C" int hk_profile_enable(hk_ctx *ctx, int on)
{
    if (!ctx) return fail(HK_E_INVALID_ARG, "NULL context");
    ctx->prof = on != 0;
    for (auto &pe : ctx->ev_used) ctx->ev_free.push_back(pe);
    ctx->ev_used.clear();
    for (double &x : ctx->prof_ms) x = 0.0;
    return HK_OK;
}

extern "C" int hk_profile_read(hk_ctx *ctx, double *out, int n)
{
    if (!ctx || !out || n < 0) return fail(HK_E_INVALID_ARG, "bad arguments");
    HIP_TRY(hipSetDevice(ctx->device));
    if (!ctx->ev_used.empty()) HIP_TRY(hipEventSynchronize(ctx->ev_used.back().e[3]));
    double acc[4] = {0, 0, 0, 0};
    for (auto &pe : ctx->ev_used) {
        float ms;
        for (int k = 0; k < 3; ++k) {
            HIP_TRY(hipEventElapsedTime(&ms, pe.e[k], pe.e[k + 1]));
            acc[k] += ms;
        }
        acc[3] += 1.0;
    }
    for (int k = 0; k < n && k < 4; ++k) out[k] = acc[k];
    return HK_OK;
}

// Fused gather, grouped compensated sums, ANOVA F-test and radius / estimate update for one set.
//
// Work decomposition: G lanes of a wavefront serve one kernel (hit point). The kernel's grid
// stencil (cells overlapping the box [x - r, x + r], grown by a rounding margin) is a list of rows
// of cells; with x fastest each row is a contiguous range of the sorted photon payload. The G lanes
// walk the concatenated rows G photons at a time (coalesced 16-byte loads), test their photon
// against the disk and accumulate into lane-private compensated sums kept in LDS. At the end the
// G partial results are combined in a fixed order (deterministic) and the kernel's epilogue runs.
//
// The test and the accumulation are decoupled: each step tests G candidates (one per lane), the
// in-disk ones are queued in LDS (lane order), and whenever a kernel has G queued photons its G
// lanes accumulate them together, so the accumulation runs with every lane busy instead of only the
// third of lanes whose candidate fell inside the disk.
//
// Light kernels use G = 16 (four kernels per wave); kernels whose stencil holds more than
// `heavy_cost` photons get a wave of their own (G = 64) and are listed first, so the longest work
// starts first. The list is rebuilt every iteration from the grid (cost = photons in the stencil).
//
// Per pair inside the disk (Sec. 3.2, Sec. 5.1):
//   y = (<x - x*, u>, <x - x*, v>)             (Eq. map-function)
//   g = annulus (2 d2 >= r2) x sector (60 degree wedges from +u)
//   S_g += psi, Q_g += psi^2                  (compensated float32 pairs)
//   flux sum += Phi (PPM) or w * beta (vertex merging, Eq. mis-weight with beta = 1)
// Epilogue per kernel: retained sums (Sec. 5.1), F in float64 (Eq. f-statistic) against the
// tabulated critical value for m = sum of J over the kept iterations, estimate update
// (Eq. progressive-VCM-estimator) with this iteration's radius, then Eq. radiusupdate.
#include <math.h>

#include "hk_fquant.h"
#include "hk_internal.h"
#include "hk_kernels.h"

namespace hk {

__device__ __forceinline__ int wave_max_i(int v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, WAVE));
    return v;
}

template <int G>
__device__ __forceinline__ uint32_t group_incl_scan(uint32_t v, int j)
{
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
        const uint32_t u = __shfl_up(v, o, G);
        if (j >= o) v += u;
    }
    return v;
}

template <int G>
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

template <int G>
__device__ __forceinline__ uint32_t group_sum_u(uint32_t v)
{
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}

// 16-byte load at a wave-uniform base plus a 32-bit byte offset (global_load with an SGPR base: no
// 64-bit address arithmetic per lane; payload planes stay below 4 GiB).
__device__ __forceinline__ float4 ld4(const float4 *base, uint32_t idx)
{
    return *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(base) + (idx << 4));
}

// Grid cells overlapping [p - r - margin, p + r + margin] on every axis; false if none.
__device__ __forceinline__ bool stencil(const SetHeader *hdr, const float p[3], float r, int c0[3], int c1[3])
{
    const float mg = fmaf(r, 1e-4f, hdr->margin_abs);
    bool any = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float f0 = floorf((p[a] - r - mg - hdr->dom_lo[a]) * hdr->cell_inv[a]);
        const float f1 = floorf((p[a] + r + mg - hdr->dom_lo[a]) * hdr->cell_inv[a]);
        const float dm = (float)(hdr->dims[a] - 1);
        any = any && (f0 <= f1) && (f1 >= 0.0f) && (f0 <= dm);
        c0[a] = (int)fminf(fmaxf(f0, 0.0f), dm);
        c1[a] = (int)fminf(fmaxf(f1, 0.0f), dm);
    }
    return any;
}

constexpr int UNROLL = 4;         // candidate loads in flight per lane
constexpr uint32_t XCD_CHUNK = 64;  // work items per XCD chunk

struct Lds {
    float4 slot[NG][WAVE];        // lane-private S, comp S, Q, comp Q per group
    float4 part[2][WAVE];         // lane-private flux pairs (R, cR, G, cG), (B, cB, -, -)
    uint32_t rs[WAVE];            // row start in the payload
    uint32_t ro[WAVE];            // row offset in the concatenation (exclusive)
    uint32_t re[WAVE];            // row end in the concatenation (inclusive scan)
    uint32_t queue[2 * WAVE];     // in-disk photons waiting for accumulation, 2 G slots per kernel
    uint32_t hist[RHIST_BINS];
};

// Per-kernel constants of one work item, held in registers by the kernel's G lanes.
struct Query {
    float p[3], nv[3], u[3], v[3];
    float r2, inv_eta, wc, cb[3];
};

// Accumulators of one lane.
struct Acc {
    float fR, cR, fG, cG, fB, cB;
    uint32_t cnt, ncand;
};

// Adds the photon pi (already inside the disk) to this lane's group sums and flux sum when it
// passes the normal-consistency test. The distance vector is recomputed from the payload with the
// same float32 operations as in the test, so the values are those the test saw.
template <bool NRM, bool VCM>
__device__ __forceinline__ void accumulate(uint32_t pi, const Query &K, float cos_min, const float4 *rA,
                                           const float4 *rB, const float4 *rC, Lds &L, int lane, Acc &c)
{
    const float4 a = ld4(rA, pi);
    const float4 f = ld4(rC, pi);
    float4 bN = make_float4(0.0f, 0.0f, 1.0f, 0.0f);
    if (NRM || VCM) bN = ld4(rB, pi);
    if (NRM) {
        const float cs = fmaf(K.nv[2], bN.z, fmaf(K.nv[1], bN.y, K.nv[0] * bN.x));
        if (!(cs >= cos_min)) return;
    }
    const float dx = K.p[0] - a.x, dy = K.p[1] - a.y, dz = K.p[2] - a.z;
    const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const float yu = fmaf(dz, K.u[2], fmaf(dy, K.u[1], dx * K.u[0]));
    const float yv = fmaf(dz, K.v[2], fmaf(dy, K.v[1], dx * K.v[0]));
    const int g = group_of(yu, yv, d2, K.r2);
    float psi, wR, wG, wB;
    if (VCM) {
        const float wl = fmaf(bN.w, INV_PI_F, f.w * K.inv_eta);
        const float w = 1.0f / ((1.0f + wl) + K.wc);
        const float yl = fmaf(0.0722f, K.cb[2] * f.z, fmaf(0.7152f, K.cb[1] * f.y, 0.2126f * (K.cb[0] * f.x)));
        psi = w * yl;
        wR = w * f.x;
        wG = w * f.y;
        wB = w * f.z;
    } else {
        psi = a.w;
        wR = f.x;
        wG = f.y;
        wB = f.z;
    }
    float4 sv = L.slot[g][lane];
    kahan(sv.x, sv.y, psi);
    kahan(sv.z, sv.w, psi * psi);
    L.slot[g][lane] = sv;
    kahan(c.fR, c.cR, wR);
    kahan(c.fG, c.cG, wG);
    kahan(c.fB, c.cB, wB);
    ++c.cnt;
}

// Each kernel's G lanes take up to G queued photons (lane j the j-th); the rest move to the front.
template <int G, bool NRM, bool VCM>
__device__ __forceinline__ void drain_once(uint32_t &qlen, int j, int base, const Query &K, float cos_min,
                                           const float4 *rA, const float4 *rB, const float4 *rC, Lds &L, int lane,
                                           Acc &c)
{
    __syncthreads();
    const uint32_t n = min(qlen, (uint32_t)G);
    if ((uint32_t)j < n) accumulate<NRM, VCM>(L.queue[2 * base + j], K, cos_min, rA, rB, rC, L, lane, c);
    const uint32_t rem = qlen - n;
    const uint32_t moved = ((uint32_t)j < rem) ? L.queue[2 * base + G + j] : 0u;
    __syncthreads();
    if ((uint32_t)j < rem) L.queue[2 * base + j] = moved;
    qlen = rem;
}

template <int G, bool NRM, bool VCM>
__device__ __forceinline__ void process(const GatherArgs &A, Lds &L, int64_t q, bool active, uint64_t &pairs_acc,
                                        uint64_t &cand_acc)
{
    const int lane = threadIdx.x;
    const int j = lane % G;
    const int base = lane - j;
    const SetHeader *hdr = A.hdr;
    const float4 *rA = A.payA, *rB = A.payB, *rC = A.payC;
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << base);
    const uint64_t below = (j == 0) ? 0ull : ((~0ull >> (64 - j)) << base);

    Query K;
    for (int a = 0; a < 3; ++a) {
        K.p[a] = 0.0f;
        K.u[a] = (a == 0) ? 1.0f : 0.0f;
        K.v[a] = (a == 1) ? 1.0f : 0.0f;
        K.nv[a] = (a == 2) ? 1.0f : 0.0f;
        K.cb[a] = 0.0f;
    }
    float r = 0.0f;
    if (active) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            K.p[a] = A.kp[a][q];
            K.u[a] = A.ku[a][q];
            K.v[a] = A.kv[a][q];
            if (NRM) K.nv[a] = A.kn[a][q];
        }
        r = A.r[q];
    }
    K.r2 = active ? r * r : -1.0f;
    K.inv_eta = 0.0f;
    K.wc = 0.0f;
    if (VCM && active) {
        const float eta = A.Jf * (PI_F * K.r2);       // n_VM / n_VC * pi r^2, n_VC = 1
        K.inv_eta = 1.0f / eta;
        K.wc = fmaf(A.cdvm[q], INV_PI_F, A.cdvcm[q] * K.inv_eta);
        K.cb[0] = A.cb[0][q];
        K.cb[1] = A.cb[1][q];
        K.cb[2] = A.cb[2][q];
    }
#pragma unroll
    for (int g = 0; g < NG; ++g) L.slot[g][lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    Acc c = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0u, 0u};
    uint32_t qlen = 0;

    int c0[3] = {0, 0, 0}, c1[3] = {0, 0, 0};
    const bool any = active && stencil(hdr, K.p, r, c0, c1);
    const int nyr = c1[1] - c0[1] + 1, nzr = c1[2] - c0[2] + 1;
    const int nrows = any ? nyr * nzr : 0;
    const uint32_t dimx = (uint32_t)hdr->dims[0], dimy = (uint32_t)hdr->dims[1];
    const int nbatch = wave_max_i((nrows + G - 1) / G);

    for (int b = 0; b < nbatch; ++b) {
        const int row = b * G + j;
        uint32_t st = 0, len = 0;
        if (row < nrows) {
            const uint32_t cy = (uint32_t)(c0[1] + row % nyr), cz = (uint32_t)(c0[2] + row / nyr);
            const uint32_t cell = (cz * dimy + cy) * dimx;
            st = A.cstart[cell + (uint32_t)c0[0]];
            len = A.cstart[cell + (uint32_t)c1[0] + 1u] - st;
        }
        const uint32_t inc = group_incl_scan<G>(len, j);
        const uint32_t total = __shfl(inc, base + G - 1, WAVE);
        __syncthreads();
        L.rs[lane] = st;
        L.ro[lane] = inc - len;
        L.re[lane] = inc;
        __syncthreads();
        const int nsteps = wave_max_i((int)((total + G - 1) / G));
        // Per-lane cursor over the concatenated rows: photon index = virtual index + delta of its row.
        // Loads are issued U steps at a time (U independent 16-byte loads in flight per lane), then
        // the U candidates are tested from registers; those inside the disk are queued.
        int cur = 0;
        uint32_t row_end = L.re[base];
        uint32_t delta = L.rs[base] - L.ro[base];
        uint32_t vi = (uint32_t)j;
        for (int s0 = 0; s0 < nsteps; s0 += UNROLL) {
            float4 a[UNROLL];
            uint32_t pis[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                pis[u] = 0xFFFFFFFFu;
                a[u] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (vi < total) {
                    while (vi >= row_end) {
                        ++cur;
                        row_end = L.re[base + cur];
                        delta = L.rs[base + cur] - L.ro[base + cur];
                    }
                    pis[u] = vi + delta;
                    a[u] = ld4(rA, pis[u]);
                }
                vi += G;
            }
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                bool in = false;
                if (pis[u] != 0xFFFFFFFFu) {
                    ++c.ncand;
                    const float dx = K.p[0] - a[u].x, dy = K.p[1] - a[u].y, dz = K.p[2] - a[u].z;
                    const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                    in = d2 < K.r2;
                }
                // queue the in-disk photons of this step in lane order
                const uint64_t m = __ballot(in);
                const uint32_t before = (uint32_t)__popcll(m & below);
                if (in) L.queue[2 * base + qlen + before] = pis[u];
                qlen += (uint32_t)__popcll(m & gmask);
                if (__ballot(qlen >= (uint32_t)G) != 0ull)
                    drain_once<G, NRM, VCM>(qlen, j, base, K, A.cos_min, rA, rB, rC, L, lane, c);
            }
        }
    }
    while (__ballot(qlen > 0u) != 0ull) drain_once<G, NRM, VCM>(qlen, j, base, K, A.cos_min, rA, rB, rC, L, lane, c);

    // Combine the G lane partials in lane order. Columns 0..11 are the groups, 12 and 13 the flux
    // pairs; lane j of the kernel combines columns j, j + G, ... (all of them in lane order).
    L.part[0][lane] = make_float4(c.fR, c.cR, c.fG, c.cG);
    L.part[1][lane] = make_float4(c.fB, c.cB, 0.0f, 0.0f);
    __syncthreads();
    constexpr int COLS = NG + 2;
    constexpr int CPL = (COLS + G - 1) / G;
    float S[CPL], cS[CPL], Q[CPL], cQ[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        const int col = j + k * G;
        S[k] = cS[k] = Q[k] = cQ[k] = 0.0f;
        if (active && col < NG) {
            S[k] = A.sq0[(size_t)(4 * col) * A.astride + q];
            cS[k] = A.sq0[(size_t)(4 * col + 1) * A.astride + q];
            Q[k] = A.sq0[(size_t)(4 * col + 2) * A.astride + q];
            cQ[k] = A.sq0[(size_t)(4 * col + 3) * A.astride + q];
        }
        if (col < COLS) {
            for (int l = 0; l < G; ++l) {
                const float4 x = (col < NG) ? L.slot[col][base + l] : L.part[col - NG][base + l];
                kahan(S[k], cS[k], x.x);
                kahan(S[k], cS[k], -x.y);
                kahan(Q[k], cQ[k], x.z);
                kahan(Q[k], cQ[k], -x.w);
            }
        }
    }
    const uint32_t cnt_q = group_sum_u<G>(c.cnt);
    const uint32_t t_new = active ? A.t[q] + 1u : 1u;
    const double m = active ? A.mprefix[A.iter] - A.mprefix[A.iter - (int)t_new] : 2.0;
    double sg[CPL], qg[CPL];
    double tl = 0.0;
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        const bool grp = j + k * G < NG;
        sg[k] = grp ? (double)S[k] - (double)cS[k] : 0.0;
        qg[k] = grp ? (double)Q[k] - (double)cQ[k] : 0.0;
        tl += sg[k];
    }
    const double tot = group_sum<G>(tl);
    double bl = 0.0, wl = 0.0;
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        if (j + k * G < NG) {
            const double d = sg[k] - tot / NG;
            bl += d * d;
            wl += qg[k] - sg[k] * sg[k] / m;
        }
    }
    const double ssb = group_sum<G>(bl) / m;
    const double ssw = group_sum<G>(wl);
    constexpr int K12 = NG / G, J12 = NG % G, K13 = (NG + 1) / G, J13 = (NG + 1) % G;
    const float flR = __shfl(S[K12] - cS[K12], base + J12, WAVE);
    const float flG = __shfl(Q[K12] - cQ[K12], base + J12, WAVE);
    const float flB = __shfl(S[K13] - cS[K13], base + J13, WAVE);

    int shrink = 0;
    if (active && j == 0) {
        const uint32_t seen = A.nseen[q] + cnt_q;
        const double F = (ssb / (NG - 1)) / (ssw / (NG * (m - 1.0)));
        const double Fc = A.fctab[t_new];
        shrink = (seen > 0u && ssw > 0.0 && m >= 2.0 && (F > Fc)) ? 1 : 0;
        // this iteration's kernel estimate with its own radius
        const float denom = A.Jf * (PI_F * K.r2);
        float eR = flR / denom, eG = flG / denom, eB = flB / denom;
        if (VCM) {
            eR = K.cb[0] * eR;
            eG = K.cb[1] * eG;
            eB = K.cb[2] * eB;
        }
        float tv[6];
#pragma unroll
        for (int cc = 0; cc < 6; ++cc) tv[cc] = A.tau0[(size_t)cc * A.astride + q];
        kahan(tv[0], tv[1], eR);
        kahan(tv[2], tv[3], eG);
        kahan(tv[4], tv[5], eB);
#pragma unroll
        for (int cc = 0; cc < 6; ++cc) A.tau0[(size_t)cc * A.astride + q] = tv[cc];
        const float rn = shrink ? fmaxf(A.k * r, A.lb) : r;
        A.r[q] = rn;
        A.t[q] = shrink ? 0u : t_new;
        A.nseen[q] = shrink ? 0u : seen;
        A.cnt[q] = cnt_q;
        A.dec[q] = shrink ? 1u : 0u;
        A.F[q] = seen > 0u ? F : (double)NAN;
        A.Fc[q] = Fc;
        atomicAdd(&L.hist[radius_bin(rn, A.r1)], 1u);
    }
    shrink = __shfl(shrink, base, WAVE);
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        const int col = j + k * G;
        if (active && col < NG) {
            A.sq0[(size_t)(4 * col) * A.astride + q] = shrink ? 0.0f : S[k];
            A.sq0[(size_t)(4 * col + 1) * A.astride + q] = shrink ? 0.0f : cS[k];
            A.sq0[(size_t)(4 * col + 2) * A.astride + q] = shrink ? 0.0f : Q[k];
            A.sq0[(size_t)(4 * col + 3) * A.astride + q] = shrink ? 0.0f : cQ[k];
        }
    }
    pairs_acc += c.cnt;
    cand_acc += c.ncand;
    __syncthreads();
}

template <bool NRM, bool VCM, int GL, int GH>
__global__ __launch_bounds__(WAVE) void gather_update_kernel(GatherArgs A)
{
    __shared__ Lds L;
    const int lane = threadIdx.x;
    L.hist[lane] = 0;
    __syncthreads();
    constexpr uint32_t KPW_L = WAVE / GL;     // light kernels per wave
    constexpr uint32_t KPW_H = WAVE / GH;     // heavy kernels per wave
    const uint32_t n_heavy = A.counts[0], n_light = A.counts[1];
    const uint32_t items_h = (n_heavy + KPW_H - 1) / KPW_H;
    const uint32_t n_items = items_h + (n_light + KPW_L - 1) / KPW_L;
    uint64_t pairs = 0, cand = 0;
    // Workgroups are dealt to the 8 XCDs round-robin. Chunk k of XCD_CHUNK consecutive items (a
    // compact patch along the Morton order) goes to XCD k mod 8, and an XCD walks its chunks in
    // order, so each XCD's L2 holds the photons of a few patches instead of the whole scene. The
    // grid is a multiple of 8 * XCD_CHUNK, which makes the map a bijection; items beyond the first
    // grid are taken in a plain stride loop.
    const uint32_t b = blockIdx.x, x = b & 7u, w = b >> 3;
    const uint32_t first = ((w / XCD_CHUNK) * 8u + x) * XCD_CHUNK + (w % XCD_CHUNK);
    for (uint32_t item = first; item < n_items; item += gridDim.x) {
        if (item < items_h) {
            const uint32_t hi = item * KPW_H + (uint32_t)(lane / GH);
            const bool act = hi < n_heavy;
            process<GH, NRM, VCM>(A, L, act ? (int64_t)A.heavy[hi] : 0, act, pairs, cand);
        } else {
            const uint32_t li = (item - items_h) * KPW_L + (uint32_t)(lane / GL);
            const bool act = li < n_light;
            process<GL, NRM, VCM>(A, L, act ? (int64_t)A.light[li] : 0, act, pairs, cand);
        }
    }
    __syncthreads();
    if (L.hist[lane]) atomicAdd(&A.hdr->rhist[lane], L.hist[lane]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        pairs += __shfl_xor(pairs, o, WAVE);
        cand += __shfl_xor(cand, o, WAVE);
    }
    if (lane == 0) {
        if (pairs) atomicAdd(&A.hdr->n_pairs, (unsigned long long)pairs);
        if (cand) atomicAdd(&A.hdr->n_cand, (unsigned long long)cand);
        if (blockIdx.x == 0) atomicAdd(&A.hdr->n_launch, 1ull);
    }
}

template <bool NRM, bool VCM>
static void launch_lanes(const GatherArgs &a, int gl, int gh, int grid, hipStream_t s)
{
#define HK_LAUNCH(GLV, GHV) gather_update_kernel<NRM, VCM, GLV, GHV><<<grid, WAVE, 0, s>>>(a)
    if (gh == 16) {
        if (gl == 4) HK_LAUNCH(4, 16);
        else if (gl == 8) HK_LAUNCH(8, 16);
        else HK_LAUNCH(16, 16);
    } else {
        if (gl == 4) HK_LAUNCH(4, 64);
        else if (gl == 8) HK_LAUNCH(8, 64);
        else HK_LAUNCH(16, 64);
    }
#undef HK_LAUNCH
}

void launch_gather(const GatherArgs &a, bool nrm, bool vcm, hipStream_t s)
{
    if (a.H <= 0) return;
    const int gl = (a.lanes_light == 4 || a.lanes_light == 8) ? a.lanes_light : 16;
    const int gh = (a.lanes_heavy == 16) ? 16 : 64;
    const int64_t per = 8 * (int64_t)XCD_CHUNK;
    const int grid = (int)(cdiv(cdiv(a.H, WAVE / gl), per) * per);
    if (nrm && vcm)
        launch_lanes<true, true>(a, gl, gh, grid, s);
    else if (nrm)
        launch_lanes<true, false>(a, gl, gh, grid, s);
    else if (vcm)
        launch_lanes<false, true>(a, gl, gh, grid, s);
    else
        launch_lanes<false, false>(a, gl, gh, grid, s);
}

// ------------------------------------------------------------------------------------------------
// work list: cost of a kernel = photons in its stencil; heavy kernels (cost > heavy_cost) first
// ------------------------------------------------------------------------------------------------

__global__ __launch_bounds__(256) void cost_kernel(ListLaunch l)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= l.H) return;
    const float p[3] = {l.kp[0][q], l.kp[1][q], l.kp[2][q]};
    int c0[3] = {0, 0, 0}, c1[3] = {0, 0, 0};
    uint32_t cost = 0;
    if (stencil(l.hdr, p, l.r[q], c0, c1)) {
        const uint32_t dimx = (uint32_t)l.hdr->dims[0], dimy = (uint32_t)l.hdr->dims[1];
        for (int cz = c0[2]; cz <= c1[2]; ++cz)
            for (int cy = c0[1]; cy <= c1[1]; ++cy) {
                const uint32_t cell = ((uint32_t)cz * dimy + (uint32_t)cy) * dimx;
                cost += l.cstart[cell + (uint32_t)c1[0] + 1u] - l.cstart[cell + (uint32_t)c0[0]];
            }
    }
    const uint32_t h = cost > l.heavy_cost ? 1u : 0u;
    l.flag[q] = h;
    l.offs[q] = h;
}

__global__ __launch_bounds__(256) void split_kernel(ListLaunch l)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= l.H) return;
    const uint32_t o = l.offs[q];
    if (l.flag[q])
        l.heavy[o] = (uint32_t)q;
    else
        l.light[(uint32_t)q - o] = (uint32_t)q;
    if (q == l.H - 1) {
        const uint32_t nh = o + l.flag[q];
        l.counts[0] = nh;
        l.counts[1] = (uint32_t)l.H - nh;
    }
}

void build_work_list(const ListLaunch &l, hipStream_t s)
{
    const int nb = (int)cdiv(l.H, 256);
    cost_kernel<<<nb, 256, 0, s>>>(l);
    excl_scan(l.offs, l.H, l.part2, s);
    split_kernel<<<nb, 256, 0, s>>>(l);
}

// ------------------------------------------------------------------------------------------------
// critical values: fctab[t] = (1 - alpha_F) quantile of F(11, 12 (m_t - 1)), m_t = J of the last t
// iterations (Sec. 3.2.2); no test (NaN) when m_t < 2
// ------------------------------------------------------------------------------------------------

__global__ __launch_bounds__(64) void fcrit_kernel(double *fctab, const double *mprefix, int iter, int t_lo,
                                                   int t_hi, double alpha)
{
    const int t = t_lo + (int)(blockIdx.x * 64 + threadIdx.x);
    if (t > t_hi) return;
    const double m = mprefix[iter] - mprefix[iter - t];
    fctab[t] = (m >= 2.0) ? f_quantile((double)(NG - 1), (double)NG * (m - 1.0), alpha) : (double)NAN;
}

void launch_fcrit(double *fctab, const double *mprefix, int iter, int t_lo, int t_hi, double alpha_f,
                  hipStream_t s)
{
    if (t_hi < t_lo) return;
    const int n = t_hi - t_lo + 1;
    fcrit_kernel<<<(int)cdiv(n, 64), 64, 0, s>>>(fctab, mprefix, iter, t_lo, t_hi, alpha_f);
}

}  // namespace hk

// Fused gather, grouped compensated sums, ANOVA F-test and radius / estimate update for a batch of
// hit-point sets.
//
// Work decomposition: G lanes of a wavefront serve one kernel (hit point). The kernel's grid
// stencil (cells overlapping the box [x - r, x + r], grown by a rounding margin) is a list of rows
// of cells; with x fastest each row is a contiguous range of the sorted photon payload, clipped to
// the x-range that can reach the disk. The G lanes walk the concatenated rows G photons at a time:
// lane j takes the candidates at positions j, j + G, ... of the concatenation, loads each one's whole
// payload (16-byte loads, four candidates in flight per lane), tests it against the disk and, when
// it is inside, adds it at once to lane-private float64 sums kept in LDS. Each lane thus sums a
// fixed subsequence of the kernel's candidates, so a kernel's sums never depend on the other kernels
// of its wave; at the end the G partial results are combined in a fixed order (deterministic) and
// the kernel's epilogue runs. Nothing waits between the test and the accumulation: the only memory
// round trips of a kernel are its rows' cell starts, its candidates and its state.
//
// Light kernels share a wave (16 lanes each as tuned); kernels whose expected candidate count
// exceeds `heavy_cost` get a whole wave and are listed first, so the longest work starts first. The
// list is rebuilt every iteration (cost = the stencil's photons in a set's first iteration, then the
// candidates tested the iteration before) and spans every set of the batch: one launch serves many
// hit-point sets of uneven size. Each lane reads its set's record (state buffer, payload and
// cell-start offsets) from a small device table, and everything that changes between iterations
// (iteration index, J, lower bound) comes from the set's state, so the launch can be replayed from a
// captured graph.
//
// Per pair inside the disk (Sec. 3.2, Sec. 5.1):
//   y = (<x - x*, u>, <x - x*, v>)             (Eq. map-function)
//   g = annulus (2 d2 >= r2) x sector (60 degree wedges from +u)
//   S_g += psi, Q_g += psi^2                  (float64: the float32 sample and its square are exact)
//   flux sum += Phi (PPM) or w * beta (vertex merging, Eq. mis-weight with beta = 1), float64
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
__device__ __forceinline__ float4 ldb(const float4 *base, uint32_t off)
{
    return *reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(base) + off);
}

constexpr int UNROLL_D = 4;       // candidates (all their payload) in flight per lane
constexpr uint32_t XCD_CHUNK = 64;  // work items per XCD chunk

// 12.5 KB per wavefront with one test channel (12 wavefronts per CU); 36.5 KB with one test per RGB
// channel.
template <int CH>
struct Lds {
    double2 slot[NG * CH][WAVE];  // lane-private sums (S, Q) per channel and group
    uint32_t dl[WAVE];            // row start, byte offset into the position plane
    uint32_t re[WAVE];            // row end (exclusive), byte offset into the position plane
};

// Per-kernel constants of one work item, held in registers by the kernel's G lanes.
struct Query {
    float p[3], nv[3], u[3], v[3];
    float r2, inv_eta, wc, cb[3];
};

// Accumulators of one lane.
struct Acc {
    double fR, fG, fB;                    // flux sums
    uint32_t cnt;
};

// The payload of one candidate: position and luminance, normal and dVM, flux and dVCM.
struct Cand {
    float4 a, b, f;
};

// A candidate is addressed by the byte offset of its payload record: (position, luminance), then
// (flux, dVCM), then (normal, dVM) when the record has it (REC = 3).
template <bool NRM, bool VCM>
__device__ __forceinline__ Cand load_cand(uint32_t off, const float4 *rec)
{
    Cand P;
    P.a = ldb(rec, off);
    P.f = ldb(rec, off + 16u);
    P.b = make_float4(0.0f, 0.0f, 1.0f, 0.0f);
    if (NRM || VCM) P.b = ldb(rec, off + 32u);
    return P;
}

// Adds a candidate found inside the disk to this lane's group sums and flux sum when it passes the
// normal-consistency test. The distance vector is recomputed with the same float32 operations as
// in the test, so the values are those the test saw. A photon that fails the normal test is added
// as zeros (an exact no-op). A float32 sample and its square are exact in float64, so each
// addition rounds once at 2^-53 of the sum: one conversion, one add and one fma per sample.
template <bool NRM, bool VCM, int CH>
__device__ __forceinline__ void accumulate(const Cand &P, const Query &K, float cos_min, Lds<CH> &L, int lane,
                                           Acc &c)
{
    const float4 a = P.a, f = P.f, bN = P.b;
    bool ok = true;
    if (NRM) {
        const float cs = fmaf(K.nv[2], bN.z, fmaf(K.nv[1], bN.y, K.nv[0] * bN.x));
        ok = cs >= cos_min;
    }
    const float dx = K.p[0] - a.x, dy = K.p[1] - a.y, dz = K.p[2] - a.z;
    const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const float yu = fmaf(dz, K.u[2], fmaf(dy, K.u[1], dx * K.u[0]));
    const float yv = fmaf(dz, K.v[2], fmaf(dy, K.v[1], dx * K.v[0]));
    const int g = group_of(yu, yv, d2, K.r2);
    // psi: the luminance test sample; pR, pG, pB: the per-channel samples; wR, wG, wB: the flux
    float psi, wR, wG, wB, pR, pG, pB;
    if (VCM) {
        const float wl = fmaf(bN.w, INV_PI_F, f.w * K.inv_eta);
        const float w = 1.0f / ((1.0f + wl) + K.wc);
        const float yl = fmaf(0.0722f, K.cb[2] * f.z, fmaf(0.7152f, K.cb[1] * f.y, 0.2126f * (K.cb[0] * f.x)));
        psi = w * yl;
        wR = w * f.x;
        wG = w * f.y;
        wB = w * f.z;
        pR = w * (K.cb[0] * f.x);
        pG = w * (K.cb[1] * f.y);
        pB = w * (K.cb[2] * f.z);
    } else {
        psi = a.w;
        wR = pR = f.x;
        wG = pG = f.y;
        wB = pB = f.z;
    }
    if (NRM && !ok) psi = wR = wG = wB = pR = pG = pB = 0.0f;
    if (CH == 1) {
        // the slot's read is issued first and the flux sums, which do not depend on it, fill its latency
        double2 sv = L.slot[g][lane];
        c.fR += (double)wR;
        c.fG += (double)wG;
        c.fB += (double)wB;
        const double x = (double)psi;
        sv.x += x;
        sv.y = fma(x, x, sv.y);
        L.slot[g][lane] = sv;
    } else {
        // one test per channel (chromatic light): the channel's sample replaces the luminance
        const float pc[3] = {pR, pG, pB};
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            double2 sv = L.slot[ch * NG + g][lane];
            const double x = (double)pc[ch];
            sv.x += x;
            sv.y = fma(x, x, sv.y);
            L.slot[ch * NG + g][lane] = sv;
        }
        c.fR += (double)wR;
        c.fG += (double)wG;
        c.fB += (double)wB;
    }
    c.cnt += ok ? 1u : 0u;
}

template <int G, bool NRM, bool VCM, int CH>
__device__ __forceinline__ void process(const BatchArgs &A, Lds<CH> &L, uint32_t entry, bool active)
{
    const int lane = threadIdx.x;
    const int j = lane % G;
    const int base = lane - j;
    // this lane's kernel: set record, then its arrays (slot k at arr + k * stride)
    const uint32_t q = entry & ((1u << Q_BITS) - 1u);
    const SetDesc D = A.desc[active ? (entry >> Q_BITS) : 0u];
    char *const arr = D.state + D.arr;
    auto fslot = [&](int k) { return reinterpret_cast<float *>(arr + (size_t)k * D.stride); };
    auto uslot = [&](int k) { return reinterpret_cast<uint32_t *>(arr + (size_t)k * D.stride); };
    auto dslot = [&](int k) { return reinterpret_cast<double *>(arr + (size_t)k * D.stride); };
    const SetHeader *hdr = reinterpret_cast<const SetHeader *>(D.state + D.hdr);
    const double *mprefix = reinterpret_cast<const double *>(D.state + D.mprefix);
    const double *fctab = reinterpret_cast<const double *>(D.state + D.fctab);
    const float *lbtab = reinterpret_cast<const float *>(D.state + D.lbtab);
    // payload records at a wave-uniform base; photon indices are global (set offset added per row)
    constexpr uint32_t RB = 16u * pay_rec(NRM || VCM);     // bytes per record
    const float4 *rec = A.pay;
    const uint32_t *cstart = A.cstart + D.cell_base;
    const int iter = active ? hdr->iter : 1;
    const float Jf = active ? hdr->Jf : 1.0f;
    const uint64_t gmask = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << base);

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
            K.p[a] = fslot(SL_POS + a)[q];
            K.u[a] = fslot(SL_U + a)[q];
            K.v[a] = fslot(SL_V + a)[q];
            if (NRM) K.nv[a] = fslot(SL_NRM + a)[q];
        }
        r = fslot(SL_R)[q];
    }
    const uint32_t t_prev = active ? uslot(SL_T)[q] : 0u;
    K.r2 = active ? r * r : -1.0f;
    K.inv_eta = 0.0f;
    K.wc = 0.0f;
    if (VCM && active) {
        const float eta = Jf * (PI_F * K.r2);         // n_VM / n_VC * pi r^2, n_VC = 1
        K.inv_eta = 1.0f / eta;
        K.wc = fmaf(fslot(SL_CDVM)[q], INV_PI_F, fslot(SL_CDVCM)[q] * K.inv_eta);
        K.cb[0] = fslot(SL_CB)[q];
        K.cb[1] = fslot(SL_CB + 1)[q];
        K.cb[2] = fslot(SL_CB + 2)[q];
    }
#pragma unroll
    for (int g = 0; g < NG * CH; ++g) L.slot[g][lane] = make_double2(0.0, 0.0);
    Acc c = {0.0, 0.0, 0.0, 0u};
    uint32_t ncand = 0;                           // candidate tests of this kernel (all row batches)

    int c0[3] = {0, 0, 0}, c1[3] = {0, 0, 0};
    const bool any = active && stencil(hdr, K.p, r, c0, c1);
    const int nyr = c1[1] - c0[1] + 1, nzr = c1[2] - c0[2] + 1;
    const int nrows = any ? nyr * nzr : 0;
    const uint32_t dimx = (uint32_t)hdr->dims[0], dimy = (uint32_t)hdr->dims[1];
    const float mg = fmaf(r, 1e-4f, hdr->margin_abs);
    const float wy = 1.0f / hdr->cell_inv[1], wz = 1.0f / hdr->cell_inv[2];
    const int nbatch = wave_max_i((nrows + G - 1) / G);

    const uint32_t sent = (A.pstride - 1u) * RB;   // byte offset of the point at infinity
    for (int b = 0; b < nbatch; ++b) {
        const int row = b * G + j;
        uint32_t st = 0, len = 0;
        int x0 = 0, x1 = 0;
        if (row < nrows &&
            row_span(hdr, K.p, r, mg, wy, wz, c0[1] + row % nyr, c0[2] + row / nyr, c0[0], c1[0], x0, x1)) {
            const uint32_t cy = (uint32_t)(c0[1] + row % nyr), cz = (uint32_t)(c0[2] + row / nyr);
            const uint32_t cell = (cz * dimy + cy) * dimx;
            const uint32_t s0 = cstart[cell + (uint32_t)x0];
            len = cstart[cell + (uint32_t)x1 + 1u] - s0;
            st = s0 + D.pay_off;
        }
        const uint32_t total = group_sum_u<G>(len);
        __syncthreads();
        L.dl[lane] = st * RB;                     // row start and end, byte offsets of records
        L.re[lane] = (st + len) * RB;
        __syncthreads();
        const int nsteps = wave_max_i((int)((total + G - 1) / G));
        ncand += total;
        // Per-lane cursor over the concatenated rows, as a byte offset of a record: lane j takes the
        // photons at positions j, j + G, ... of the concatenation. Passing a row's end carries the
        // overshoot into the next row; past the last non-empty row the cursor rests on the point at
        // infinity. The payloads of U steps are loaded together (U candidates in flight per lane),
        // then the U candidates are tested from registers and those inside the disk accumulated.
        const uint64_t nonempty = __ballot(len > 0u) & gmask;
        const int last = nonempty ? (63 - __clzll((long long)nonempty)) - base : -1;
        int cur = 0;
        uint32_t end = L.re[base];
        uint32_t off = L.dl[base] + (uint32_t)j * RB;
        uint32_t stride = (uint32_t)G * RB;
        for (int s0 = 0; s0 < nsteps; s0 += UNROLL_D) {
            Cand P[UNROLL_D];
#pragma unroll
            for (int u = 0; u < UNROLL_D; ++u) {
                while (off >= end) {
                    if (++cur > last) {
                        off = sent;
                        stride = 0u;
                        end = 0xFFFFFFFFu;
                    } else {
                        off = (off - end) + L.dl[base + cur];
                        end = L.re[base + cur];
                    }
                }
                P[u] = load_cand<NRM, VCM>(off, rec);
                off += stride;
            }
#pragma unroll
            for (int u = 0; u < UNROLL_D; ++u) {
                const float dx = K.p[0] - P[u].a.x, dy = K.p[1] - P[u].a.y, dz = K.p[2] - P[u].a.z;
                const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                if (d2 < K.r2) accumulate<NRM, VCM, CH>(P[u], K, A.cos_min, L, lane, c);
            }
        }
    }
    // The epilogue's state reads: the retained sums of the lane's columns, the kept-iteration
    // count's J sums and critical value, and (first lane) the photons seen and the running estimate.
    constexpr int COLS = NG * CH;                 // column = channel * NG + group
    constexpr int CPL = (COLS + G - 1) / G;
    double2 *const sq2 = reinterpret_cast<double2 *>(fslot(SL_SQ));   // per hit point, COLS (S, Q)
    double S[CPL], Q[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        const int col = j + k * G;
        S[k] = Q[k] = 0.0;
        if (active && col < COLS) {
            const double2 x = sq2[(size_t)q * COLS + col];
            S[k] = x.x;
            Q[k] = x.y;
        }
    }
    const uint32_t t_new = t_prev + 1u;
    const double m = active ? mprefix[iter] - mprefix[iter - (int)t_new] : 2.0;
    const double inv_m = 1.0 / m;                 // one float64 division per lane, products after it
    const bool lead = active && j == 0;
    const double Fc = lead ? fctab[t_new] : 0.0;
    const uint32_t seen_prev = lead ? uslot(SL_NSEEN)[q] : 0u;
    float tv[6];
#pragma unroll
    for (int cc = 0; cc < 6; ++cc) tv[cc] = lead ? fslot(SL_TAU + cc)[q] : 0.0f;

    __syncthreads();

    // Combine the G lane partials: lane j of the kernel combines groups j, j + G, ... from LDS in
    // lane order (a whole-wavefront kernel: four lanes per group, 16 partials each, then a
    // butterfly); the flux sums are folded across the kernel's lanes by a butterfly (both partners
    // of a step add the same two values, so they hold the same sum).
    const double fR = group_sum<G>(c.fR), fG = group_sum<G>(c.fG), fB = group_sum<G>(c.fB);
    if constexpr (G == WAVE && COLS <= 16) {
        // the retained sums sit in lanes 0..COLS-1 (zero elsewhere) and enter once
        const int col = j & 15, sub = j >> 4;
        if (col < COLS) {
            for (int l = 0; l < 16; ++l) {
                const double2 x = L.slot[col][base + sub * 16 + l];
                S[0] += x.x;
                Q[0] += x.y;
            }
        }
#pragma unroll
        for (int o = 16; o < WAVE; o <<= 1) {
            S[0] += __shfl_xor(S[0], o, WAVE);
            Q[0] += __shfl_xor(Q[0], o, WAVE);
        }
    } else {
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            const int col = j + k * G;
            if (col < COLS) {
                for (int l = 0; l < G; ++l) {
                    const double2 x = L.slot[col][base + l];
                    S[k] += x.x;
                    Q[k] += x.y;
                }
            }
        }
    }
    const uint32_t cnt_q = group_sum_u<G>(c.cnt);
    // per channel: total, between- and within-group sums of squares (Eq. f-statistic), the lane's
    // columns first, then summed over the kernel's lanes
    double sg[CPL], qg[CPL];
    double tl[CH], bl[CH], wl[CH], ssb[CH], ssw[CH];
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) tl[ch] = bl[ch] = wl[ch] = 0.0;
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        const int col = j + k * G;
        const bool grp = col < COLS;
        sg[k] = grp ? S[k] : 0.0;
        qg[k] = grp ? Q[k] : 0.0;
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) tl[ch] += (grp && col / NG == ch) ? sg[k] : 0.0;
    }
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) tl[ch] = group_sum<G>(tl[ch]);
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        const int col = j + k * G;
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) {
            if (col < COLS && col / NG == ch) {
                const double d = sg[k] - tl[ch] * (1.0 / NG);
                bl[ch] += d * d;
                wl[ch] += qg[k] - sg[k] * sg[k] * inv_m;
            }
        }
    }
#pragma unroll
    for (int ch = 0; ch < CH; ++ch) {
        ssb[ch] = group_sum<G>(bl[ch]) * inv_m;
        ssw[ch] = group_sum<G>(wl[ch]);
    }
    const float flR = (float)fR, flG = (float)fG, flB = (float)fB;

    int shrink = 0;
    if (active && j == 0) {
        const uint32_t seen = seen_prev + cnt_q;
        // one test per channel: reject when any channel rejects; report the largest F
        double F = (double)NAN;
#pragma unroll
        for (int ch = 0; ch < CH; ++ch) {
            // (ssb / (NG - 1)) / (ssw / (NG (m - 1))) with one division
            const double Fch = (ssb[ch] * (NG * (m - 1.0))) / ((double)(NG - 1) * ssw[ch]);
            if (seen > 0u && ssw[ch] > 0.0 && m >= 2.0 && Fch > Fc) shrink = 1;
            F = fmax(F, Fch);
        }
        // this iteration's kernel estimate with its own radius
        const float denom = Jf * (PI_F * K.r2);
        float eR = flR / denom, eG = flG / denom, eB = flB / denom;
        if (VCM) {
            eR = K.cb[0] * eR;
            eG = K.cb[1] * eG;
            eB = K.cb[2] * eB;
        }
        acc2(tv[0], tv[1], eR);
        acc2(tv[2], tv[3], eG);
        acc2(tv[4], tv[5], eB);
#pragma unroll
        for (int cc = 0; cc < 6; ++cc) fslot(SL_TAU + cc)[q] = tv[cc];
        const float rn = shrink ? fmaxf(A.k * r, lbtab[iter + 1]) : r;
        fslot(SL_R)[q] = rn;
        uslot(SL_T)[q] = shrink ? 0u : t_new;
        uslot(SL_NSEEN)[q] = shrink ? 0u : seen;
        uslot(SL_CNT)[q] = cnt_q;
        uslot(SL_DEC)[q] = shrink ? 1u : 0u;
        uslot(SL_CAND)[q] = ncand;
        dslot(SL_F)[q] = seen > 0u ? F : (double)NAN;
        dslot(SL_FC)[q] = Fc;
    }
    shrink = __shfl(shrink, base, WAVE);
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
        const int col = j + k * G;
        if (active && col < COLS)
            sq2[(size_t)q * COLS + col] = shrink ? make_double2(0.0, 0.0) : make_double2(S[k], Q[k]);
    }
    __syncthreads();
}

template <bool NRM, bool VCM, int CH, int GL, int GH>
__global__ __launch_bounds__(WAVE) void gather_update_kernel(BatchArgs A)
{
    __shared__ Lds<CH> L;
    const int lane = threadIdx.x;
    constexpr uint32_t KPW_L = WAVE / GL;     // light kernels per wave
    constexpr uint32_t KPW_H = WAVE / GH;     // heavy kernels per wave
    const uint32_t n_heavy = A.counts[0], n_light = A.counts[1];
    // heavy items padded to whole XCD chunks, so that each chunk of light items is one cost-sorted
    // run of the light list (a compact patch)
    const uint32_t items_h = ((n_heavy + KPW_H - 1) / KPW_H + XCD_CHUNK - 1) / XCD_CHUNK * XCD_CHUNK;
    const uint32_t n_items = items_h + (n_light + KPW_L - 1) / KPW_L;
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
            process<GH, NRM, VCM, CH>(A, L, act ? A.heavy[hi] : 0u, act);
        } else {
            const uint32_t li = (item - items_h) * KPW_L + (uint32_t)(lane / GL);
            const bool act = li < n_light;
            process<GL, NRM, VCM, CH>(A, L, act ? A.light[li] : 0u, act);
        }
    }
}

template <bool NRM, bool VCM, int CH>
static void launch_lanes(const BatchArgs &a, int gl, int gh, int grid, hipStream_t s)
{
#define HK_LAUNCH(GLV, GHV) gather_update_kernel<NRM, VCM, CH, GLV, GHV><<<grid, WAVE, 0, s>>>(a)
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

template <int CH>
static void launch_modes(const BatchArgs &a, bool nrm, bool vcm, int gl, int gh, int grid, hipStream_t s)
{
    if (nrm && vcm)
        launch_lanes<true, true, CH>(a, gl, gh, grid, s);
    else if (nrm)
        launch_lanes<true, false, CH>(a, gl, gh, grid, s);
    else if (vcm)
        launch_lanes<false, true, CH>(a, gl, gh, grid, s);
    else
        launch_lanes<false, false, CH>(a, gl, gh, grid, s);
}

void launch_gather(const BatchArgs &a, int64_t h_total, bool nrm, bool vcm, int nch, hipStream_t s)
{
    if (h_total <= 0) return;
    const int gl = (a.lanes_light == 4 || a.lanes_light == 8) ? a.lanes_light : 16;
    const int gh = (a.lanes_heavy == 16) ? 16 : 64;
    const int64_t per = 8 * (int64_t)XCD_CHUNK;
    const int grid = (int)(cdiv(cdiv(h_total, WAVE / gl), per) * per);
    if (nch == 3)
        launch_modes<3>(a, nrm, vcm, gl, gh, grid, s);
    else
        launch_modes<1>(a, nrm, vcm, gl, gh, grid, s);
}

// ------------------------------------------------------------------------------------------------
// work list: cost of a kernel = photons in its stencil; heavy kernels (cost > heavy_cost) first.
// Each set writes its kernels' flags and entries at its offset in the batch; one scan and one split
// over the whole batch give the heavy list and the light list, both in set order.
// ------------------------------------------------------------------------------------------------

__device__ __forceinline__ void cost_items(const ListLaunch &l, int64_t q0)
{
    const bool in = q0 < l.H;
    const int64_t q = in ? q0 : l.H - 1;
    const float p[3] = {l.kp[0][q], l.kp[1][q], l.kp[2][q]};
    int c0[3] = {0, 0, 0}, c1[3] = {0, 0, 0};
    uint32_t cost = 0;
    // the set's first iteration (the plan has advanced the count to 1) counts the stencil's photons;
    // later ones take the estimate, decided on the device so that a captured graph does the same
    if (l.hdr->iter > 1) {
        // the last iteration's candidate tests, scaled by the area ratio k^2 where the radius shrank
        const uint32_t prev = l.cand[q];
        cost = l.dec[q] ? (uint32_t)((float)prev * l.k2) : prev;
    } else if (in && stencil(l.hdr, p, l.r[q], c0, c1)) {
        const uint32_t dimx = (uint32_t)l.hdr->dims[0], dimy = (uint32_t)l.hdr->dims[1];
        const float rq = l.r[q];
        const float mg = fmaf(rq, 1e-4f, l.hdr->margin_abs);
        const float wy = 1.0f / l.hdr->cell_inv[1], wz = 1.0f / l.hdr->cell_inv[2];
        for (int cz = c0[2]; cz <= c1[2]; ++cz)
            for (int cy = c0[1]; cy <= c1[1]; ++cy) {
                int x0, x1;
                if (!row_span(l.hdr, p, rq, mg, wy, wz, cy, cz, c0[0], c1[0], x0, x1)) continue;
                const uint32_t cell = ((uint32_t)cz * dimy + (uint32_t)cy) * dimx;
                cost += l.cstart[cell + (uint32_t)x1 + 1u] - l.cstart[cell + (uint32_t)x0];
            }
    }
    const uint32_t h = cost > l.heavy_cost ? 1u : 0u;
    if (in) {
        l.flag[q] = cost;
        l.ids[q] = (l.set_slot << Q_BITS) | (uint32_t)q;
    }
    // heavy kernels per tile of SPLIT_TILE entries of the batch's work list (a wavefront's entries
    // touch at most two tiles): one atomic per wavefront and tile
    {
        const uint32_t g = l.q_base + (uint32_t)q;
        const uint32_t tile = g / SPLIT_TILE;
        const uint32_t t0 = __shfl(tile, 0, WAVE);
        const uint64_t m0 = __ballot(in && h && tile == t0), m1 = __ballot(in && h && tile != t0);
        if ((threadIdx.x & (WAVE - 1)) == 0 && m0) atomicAdd(&l.tile_heavy[t0], (uint32_t)__popcll(m0));
        if (in && h && tile != t0 && (uint32_t)__popcll(m1 & ((1ull << (threadIdx.x & (WAVE - 1))) - 1ull)) == 0u)
            atomicAdd(&l.tile_heavy[tile], (uint32_t)__popcll(m1));
    }
}

// One launch over the sets of a gather phase: block b serves 256 kernels of the set block_set picks.
__global__ __launch_bounds__(256) void cost_batch_kernel(CostBatch c, SetBlocks B)
{
    const int i = block_set(B, blockIdx.x);
    const int k = c.k0 + i;
    const SetDesc D = c.desc[k];
    const char *arr = D.state + D.arr;
    auto fs = [&](int slot) { return reinterpret_cast<const float *>(arr + (size_t)slot * D.stride); };
    auto us = [&](int slot) { return reinterpret_cast<const uint32_t *>(arr + (size_t)slot * D.stride); };
    ListLaunch l{};
    l.H = D.H;
    l.hdr = reinterpret_cast<SetHeader *>(D.state + D.hdr);
    l.cstart = c.cstart + D.cell_base;
    for (int a = 0; a < 3; ++a) l.kp[a] = fs(SL_POS + a);
    l.r = fs(SL_R);
    l.cand = us(SL_CAND);
    l.dec = us(SL_DEC);
    l.k2 = c.k2;
    l.heavy_cost = c.heavy_cost;
    l.set_slot = (uint32_t)k;
    l.q_base = D.q_off - c.q0;
    l.flag = c.flag + D.q_off;
    l.ids = c.ids + D.q_off;
    l.tile_heavy = c.tile_heavy;
    cost_items(l, (int64_t)(blockIdx.x - B.pre[i]) * 256 + threadIdx.x);
}

void launch_cost_batch(const CostBatch &c, const uint32_t *H, hipStream_t s)
{
    SetBlocks B{};
    B.n = c.k1 - c.k0;
    if (B.n <= 0) return;
    uint32_t nblk = 0;
    for (int i = 0; i < B.n; ++i) {
        B.pre[i] = nblk;
        nblk += (uint32_t)cdiv(H[c.k0 + i], 256);
    }
    B.pre[B.n] = nblk;
    if (nblk == 0) return;
    cost_batch_kernel<<<(int)nblk, 256, 0, s>>>(c, B);
}

// Stable partition of the batch's work list, heavy kernels first, in kernel order within each list
// (the Morton order of each set, sets in batch order): the order keeps neighbouring kernels together,
// which the gather's cache reuse depends on. One block per tile of SPLIT_TILE entries: the heavy
// kernels of the earlier tiles (counted by the cost kernels) give the tile's offset, a block scan
// the ranks inside it.
__global__ __launch_bounds__(256) void split_kernel(const uint32_t *cost, const uint32_t *ids, int64_t n,
                                                    uint32_t heavy_cost, const uint32_t *tile_heavy, uint32_t *heavy,
                                                    uint32_t *light, uint32_t *lcost, uint32_t *counts,
                                                    float4 *sentinel)
{
    constexpr int PER = SPLIT_TILE / 256;
    // the payload's last position entry: a point at infinity, the gather's stand-in once a lane has
    // walked past its kernel's last row (outside every disk, never accumulated)
    if (blockIdx.x == 0 && threadIdx.x == 0) *sentinel = make_float4(INFINITY, INFINITY, INFINITY, 0.0f);
    // heavy entries of the tiles before this one, summed by the whole block
    uint32_t hb = 0;
    for (uint32_t t = threadIdx.x; t < blockIdx.x; t += 256) hb += tile_heavy[t];
    uint32_t before;
    block_excl_scan(hb, &before);
    const int64_t base = (int64_t)blockIdx.x * SPLIT_TILE + (int64_t)threadIdx.x * PER;
    // a thread's PER entries as 16-byte words when they are all present and both arrays are 16-byte
    // aligned (a set's entries begin at any 4-byte offset of the batch's arrays)
    const bool vec = base + PER <= n && ((reinterpret_cast<uintptr_t>(cost) | reinterpret_cast<uintptr_t>(ids)) & 15u) == 0;
    uint32_t cv[PER], iv[PER];
    if (vec) {
#pragma unroll
        for (int i = 0; i < PER; i += 4) {
            const uint4 x = *reinterpret_cast<const uint4 *>(cost + base + i);
            const uint4 y = *reinterpret_cast<const uint4 *>(ids + base + i);
            cv[i] = x.x, cv[i + 1] = x.y, cv[i + 2] = x.z, cv[i + 3] = x.w;
            iv[i] = y.x, iv[i + 1] = y.y, iv[i + 2] = y.z, iv[i + 3] = y.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            cv[i] = base + i < n ? cost[base + i] : 0u;
            iv[i] = base + i < n ? ids[base + i] : 0u;
        }
    }
    uint32_t f[PER];
    uint32_t c = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        f[i] = (base + i < n && cv[i] > heavy_cost) ? 1u : 0u;
        c += f[i];
    }
    uint32_t tot;
    const uint32_t ex = block_excl_scan(c, &tot);
    uint32_t o = before + ex;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int64_t q = base + i;
        if (q < n) {
            if (f[i]) {
                heavy[o] = iv[i];
            } else {
                light[(uint32_t)q - o] = iv[i];
                lcost[(uint32_t)q - o] = cv[i];
            }
        }
        o += f[i];
    }
    if ((int64_t)(blockIdx.x + 1) * SPLIT_TILE >= n && threadIdx.x == 0) {
        const uint32_t nh = before + tot;
        counts[0] = nh;
        counts[1] = (uint32_t)n - nh;
    }
}

// The light list in runs of LSORT entries sorted by expected cost (ties by position): a wavefront's
// kernels then carry similar work, while a run (a compact patch of the Morton order, as many
// wavefronts as an XCD chunk) keeps its cache locality. Bitonic sort of (cost, position) keys.
constexpr int LSORT = 256;
static_assert(LSORT == XCD_CHUNK * (WAVE / 16), "a sorted run is one XCD chunk of 16-lane light items");

__global__ __launch_bounds__(LSORT) void light_sort_kernel(uint32_t *light, const uint32_t *lcost,
                                                           const uint32_t *counts)
{
    __shared__ uint64_t key[LSORT];
    const uint32_t n = counts[1];
    const uint32_t b0 = blockIdx.x * LSORT;
    if (b0 >= n) return;
    const int t = threadIdx.x;
    const uint32_t i = b0 + (uint32_t)t;
    key[t] = (i < n) ? (((uint64_t)lcost[i] << 40) | ((uint64_t)t << 32) | light[i]) : ~0ull;
    __syncthreads();
    for (int k = 2; k <= LSORT; k <<= 1) {
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            const int p = t ^ jj;
            if (p > t) {
                const uint64_t a = key[t], b = key[p];
                const bool up = (t & k) == 0;
                if ((a > b) == up) {
                    key[t] = b;
                    key[p] = a;
                }
            }
            __syncthreads();
        }
    }
    if (i < n) light[i] = (uint32_t)key[t];
}

void launch_split(uint32_t *cost, uint32_t *ids, int64_t n, uint32_t heavy_cost, const uint32_t *tile_heavy,
                  uint32_t *heavy, uint32_t *light, uint32_t *lcost, uint32_t *counts, float4 *sentinel,
                  hipStream_t s)
{
    if (n <= 0) return;
    split_kernel<<<(int)cdiv(n, SPLIT_TILE), 256, 0, s>>>(cost, ids, n, heavy_cost, tile_heavy, heavy, light, lcost,
                                                          counts, sentinel);
    light_sort_kernel<<<(int)cdiv(n, LSORT), LSORT, 0, s>>>(light, lcost, counts);
}

// ------------------------------------------------------------------------------------------------
// after the update: per set, the histogram of the new radii (the next plan's cell size) and the
// in-disk pairs and candidate tests of the iteration. Every block serves TALLY_PER_BLOCK kernels of
// one set, tallies them in LDS and adds its nonzero bins and totals to the set's header.
// ------------------------------------------------------------------------------------------------

constexpr int TALLY_PER_BLOCK = 4096;

__global__ __launch_bounds__(256) void tally_kernel(const SetDesc *desc, SetBlocks B)
{
    __shared__ uint32_t hist[RHIST_BINS];
    __shared__ unsigned long long pairs, cands;
    const int k = block_set(B, blockIdx.x);
    const SetDesc D = desc[k];
    SetHeader *h = reinterpret_cast<SetHeader *>(D.state + D.hdr);
    const float r1 = h->r1;
    const char *arr = D.state + D.arr;
    const float *rr = reinterpret_cast<const float *>(arr + (size_t)SL_R * D.stride);
    const uint32_t *cnt = reinterpret_cast<const uint32_t *>(arr + (size_t)SL_CNT * D.stride);
    const uint32_t *cand = reinterpret_cast<const uint32_t *>(arr + (size_t)SL_CAND * D.stride);
    const int64_t q0 = (int64_t)(blockIdx.x - B.pre[k]) * TALLY_PER_BLOCK;
    const int64_t q1 = min((int64_t)D.H, q0 + (int64_t)TALLY_PER_BLOCK);
    if (threadIdx.x < RHIST_BINS) hist[threadIdx.x] = 0u;
    if (threadIdx.x == 0) pairs = cands = 0ull;
    __syncthreads();
    unsigned long long acc = 0, accc = 0;
    for (int64_t q = q0 + threadIdx.x; q < q1; q += 256) {
        acc += cnt[q];
        accc += cand[q];
        atomicAdd(&hist[radius_bin(rr[q], r1)], 1u);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        acc += __shfl_xor(acc, o, WAVE);
        accc += __shfl_xor(accc, o, WAVE);
    }
    if ((threadIdx.x & (WAVE - 1)) == 0 && acc) atomicAdd(&pairs, acc);
    if ((threadIdx.x & (WAVE - 1)) == 0 && accc) atomicAdd(&cands, accc);
    __syncthreads();
    if (threadIdx.x < RHIST_BINS && hist[threadIdx.x]) atomicAdd(&h->rhist[threadIdx.x], hist[threadIdx.x]);
    if (threadIdx.x == 0 && pairs) atomicAdd(&h->n_pairs, pairs);
    if (threadIdx.x == 0 && cands) atomicAdd(&h->n_cand, cands);
}

void launch_tally(const SetDesc *desc, const uint32_t *H, int nb, hipStream_t s)
{
    SetBlocks B{};
    B.n = nb;
    uint32_t nblk = 0;
    for (int k = 0; k < nb; ++k) {
        B.pre[k] = nblk;
        nblk += (uint32_t)cdiv(H[k], TALLY_PER_BLOCK);
    }
    B.pre[nb] = nblk;
    if (nblk == 0) return;
    tally_kernel<<<(int)nblk, 256, 0, s>>>(desc, B);
}

// ------------------------------------------------------------------------------------------------
// critical values: fctab[t] = (1 - alpha_F) quantile of F(11, 12 (m_t - 1)), m_t = J of the last t
// iterations (Sec. 3.2.2); no test (NaN) when m_t < 2. The iteration index is read from the set
// header (advanced by the plan kernel). With `all` every t = 1..iter is recomputed (J changed at
// some point); otherwise only t = iter is new, since with a constant J the earlier entries hold.
// ------------------------------------------------------------------------------------------------

// One launch for a batch: blockIdx.y is the set, blockIdx.x the block of t values (all[k]) or 0.
struct FcritBatch {
    const SetDesc *desc;
    double alpha;
    uint8_t all[MAX_BATCH];
};

__global__ __launch_bounds__(64) void fcrit_kernel(FcritBatch F)
{
    const SetDesc D = F.desc[blockIdx.y];
    const SetHeader *hdr = reinterpret_cast<const SetHeader *>(D.state + D.hdr);
    double *fctab = reinterpret_cast<double *>(D.state + D.fctab);
    const double *mprefix = reinterpret_cast<const double *>(D.state + D.mprefix);
    const int all = F.all[blockIdx.y];
    const int iter = hdr->iter;
    const int t = all ? 1 + (int)(blockIdx.x * 64 + threadIdx.x) : iter;
    if (t > iter || (!all && (blockIdx.x != 0 || threadIdx.x != 0))) return;
    const double m = mprefix[iter] - mprefix[iter - t];
    fctab[t] = (m >= 2.0) ? f_quantile((double)(NG - 1), (double)NG * (m - 1.0), F.alpha) : (double)NAN;
}

void launch_fcrit(const SetDesc *desc, int nb, const uint8_t *all, int max_iters, double alpha_f, hipStream_t s)
{
    FcritBatch F{};
    F.desc = desc;
    F.alpha = alpha_f;
    bool any_all = false;
    for (int k = 0; k < nb && k < MAX_BATCH; ++k) {
        F.all[k] = all[k];
        any_all = any_all || all[k];
    }
    const int nx = any_all ? (int)cdiv(max_iters, 64) : 1;
    fcrit_kernel<<<dim3(nx, nb), 64, 0, s>>>(F);
}

}  // namespace hk

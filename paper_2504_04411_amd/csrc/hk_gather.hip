// Fused gather, grouped compensated sums, ANOVA F-test and radius / estimate update for one set.
//
// Work decomposition: G lanes of a wavefront serve one kernel (hit point). The kernel's grid
// stencil (cells overlapping the box [x - r, x + r], grown by a rounding margin) is a list of rows
// of cells; with x fastest each row is a contiguous range of the sorted photon payload. The G lanes
// walk the concatenated rows G photons at a time (coalesced 16-byte loads), test their photon
// against the disk and accumulate into lane-private compensated sums kept in LDS. At the end the
// G partial results are combined in a fixed order (deterministic) and the kernel's epilogue runs.
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

struct Lds {
    float4 slot[NG][WAVE];        // lane-private S, comp S, Q, comp Q per group
    float4 part[2][WAVE];         // lane-private flux pairs (R, cR, G, cG), (B, cB, -, -)
    uint32_t rs[WAVE];            // row start in the payload
    uint32_t ro[WAVE];            // row offset in the concatenation (exclusive)
    uint32_t re[WAVE];            // row end in the concatenation (inclusive scan)
    uint32_t hist[RHIST_BINS];
};

template <int G, bool NRM, bool VCM>
__device__ __forceinline__ void process(const GatherArgs &A, Lds &L, int64_t q, bool active, uint64_t &pairs_acc,
                                        uint64_t &cand_acc)
{
    const int lane = threadIdx.x;
    const int j = lane % G;
    const int base = lane - j;
    const SetHeader *hdr = A.hdr;
    const float4 *rA = A.payA, *rB = A.payB, *rC = A.payC;

    float p[3] = {0.0f, 0.0f, 0.0f}, nv[3] = {0.0f, 0.0f, 1.0f}, u[3] = {1.0f, 0.0f, 0.0f}, v[3] = {0.0f, 1.0f, 0.0f};
    float r = 0.0f;
    if (active) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            p[a] = A.kp[a][q];
            u[a] = A.ku[a][q];
            v[a] = A.kv[a][q];
            if (NRM) nv[a] = A.kn[a][q];
        }
        r = A.r[q];
    }
    const float r2 = active ? r * r : -1.0f;
    float inv_eta = 0.0f, wc = 0.0f, cbR = 0.0f, cbG = 0.0f, cbB = 0.0f;
    if (VCM && active) {
        const float eta = A.Jf * (PI_F * r2);       // n_VM / n_VC * pi r^2, n_VC = 1
        inv_eta = 1.0f / eta;
        wc = fmaf(A.cdvm[q], INV_PI_F, A.cdvcm[q] * inv_eta);
        cbR = A.cb[0][q];
        cbG = A.cb[1][q];
        cbB = A.cb[2][q];
    }
#pragma unroll
    for (int g = 0; g < NG; ++g) L.slot[g][lane] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float fR = 0.0f, cR = 0.0f, fG = 0.0f, cG = 0.0f, fB = 0.0f, cB = 0.0f;
    uint32_t cnt = 0, ncand = 0;

    int c0[3] = {0, 0, 0}, c1[3] = {0, 0, 0};
    const bool any = active && stencil(hdr, p, r, c0, c1);
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
        // per-lane cursor over the concatenated rows: photon index = virtual index + delta of its row
        int cur = 0;
        uint32_t row_end = L.re[base];
        uint32_t delta = L.rs[base] - L.ro[base];
        uint32_t vi = (uint32_t)j;
        bool val_n = vi < total;
        uint32_t pi_n = 0;
        float4 a_n = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (val_n) {
            while (vi >= row_end) {
                ++cur;
                row_end = L.re[base + cur];
                delta = L.rs[base + cur] - L.ro[base + cur];
            }
            pi_n = vi + delta;
            a_n = ld4(rA, pi_n);
        }
        for (int s = 0; s < nsteps; ++s) {
            const bool val = val_n;
            const uint32_t pi = pi_n;
            const float4 a = a_n;
            vi += G;
            val_n = vi < total;
            if (val_n) {                      // issue the next photon's load before using this one
                while (vi >= row_end) {
                    ++cur;
                    row_end = L.re[base + cur];
                    delta = L.rs[base + cur] - L.ro[base + cur];
                }
                pi_n = vi + delta;
                a_n = ld4(rA, pi_n);
            }
            if (val) {
                ++ncand;
                const float dx = p[0] - a.x, dy = p[1] - a.y, dz = p[2] - a.z;
                const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                bool in = d2 < r2;
                float4 bN = make_float4(0.0f, 0.0f, 1.0f, 0.0f);
                if (NRM || VCM) {
                    if (in) bN = ld4(rB, pi);
                }
                if (NRM) {
                    const float c = fmaf(nv[2], bN.z, fmaf(nv[1], bN.y, nv[0] * bN.x));
                    in = in && (c >= A.cos_min);
                }
                if (in) {
                    const float4 f = ld4(rC, pi);
                    const float yu = fmaf(dz, u[2], fmaf(dy, u[1], dx * u[0]));
                    const float yv = fmaf(dz, v[2], fmaf(dy, v[1], dx * v[0]));
                    const int g = group_of(yu, yv, d2, r2);
                    float psi, wR, wG, wB;
                    if (VCM) {
                        const float wl = fmaf(bN.w, INV_PI_F, f.w * inv_eta);
                        const float w = 1.0f / ((1.0f + wl) + wc);
                        const float yl = fmaf(0.0722f, cbB * f.z, fmaf(0.7152f, cbG * f.y, 0.2126f * (cbR * f.x)));
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
                    kahan(fR, cR, wR);
                    kahan(fG, cG, wG);
                    kahan(fB, cB, wB);
                    ++cnt;
                }
            }
        }
    }

    // combine the G lane partials in lane order: lane j < 12 sums group j, lanes 12 and 13 the flux
    L.part[0][lane] = make_float4(fR, cR, fG, cG);
    L.part[1][lane] = make_float4(fB, cB, 0.0f, 0.0f);
    __syncthreads();
    float S = 0.0f, cS = 0.0f, Q = 0.0f, cQ = 0.0f;
    if (active && j < NG) {
        S = A.sq[4 * j][q];
        cS = A.sq[4 * j + 1][q];
        Q = A.sq[4 * j + 2][q];
        cQ = A.sq[4 * j + 3][q];
    }
    if (j < NG + 2) {
        for (int l = 0; l < G; ++l) {
            const float4 x = (j < NG) ? L.slot[j][base + l] : L.part[j - NG][base + l];
            kahan(S, cS, x.x);
            kahan(S, cS, -x.y);
            kahan(Q, cQ, x.z);
            kahan(Q, cQ, -x.w);
        }
    }
    const uint32_t cnt_q = group_sum_u<G>(cnt);
    const uint32_t t_new = active ? A.t[q] + 1u : 1u;
    const double m = active ? A.mprefix[A.iter] - A.mprefix[A.iter - (int)t_new] : 2.0;
    const double Sg = (j < NG) ? (double)S - (double)cS : 0.0;
    const double Qg = (j < NG) ? (double)Q - (double)cQ : 0.0;
    const double tot = group_sum<G>(Sg);
    const double dmean = (j < NG) ? Sg - tot / NG : 0.0;
    const double ssb = group_sum<G>(dmean * dmean) / m;
    const double ssw = group_sum<G>((j < NG) ? Qg - Sg * Sg / m : 0.0);
    const float flR = __shfl(S - cS, base + NG, WAVE);
    const float flG = __shfl(Q - cQ, base + NG, WAVE);
    const float flB = __shfl(S - cS, base + NG + 1, WAVE);

    int shrink = 0;
    if (active && j == 0) {
        const uint32_t seen = A.nseen[q] + cnt_q;
        const double F = (ssb / (NG - 1)) / (ssw / (NG * (m - 1.0)));
        const double Fc = A.fctab[t_new];
        shrink = (seen > 0u && ssw > 0.0 && m >= 2.0 && (F > Fc)) ? 1 : 0;
        // this iteration's kernel estimate with its own radius
        const float denom = A.Jf * (PI_F * r2);
        float eR = flR / denom, eG = flG / denom, eB = flB / denom;
        if (VCM) {
            eR = cbR * eR;
            eG = cbG * eG;
            eB = cbB * eB;
        }
        float tv[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) tv[c] = A.tau[c][q];
        kahan(tv[0], tv[1], eR);
        kahan(tv[2], tv[3], eG);
        kahan(tv[4], tv[5], eB);
#pragma unroll
        for (int c = 0; c < 6; ++c) A.tau[c][q] = tv[c];
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
    if (active && j < NG) {
        A.sq[4 * j][q] = shrink ? 0.0f : S;
        A.sq[4 * j + 1][q] = shrink ? 0.0f : cS;
        A.sq[4 * j + 2][q] = shrink ? 0.0f : Q;
        A.sq[4 * j + 3][q] = shrink ? 0.0f : cQ;
    }
    pairs_acc += cnt;
    cand_acc += ncand;
    __syncthreads();
}

template <bool NRM, bool VCM>
__global__ __launch_bounds__(WAVE) void gather_update_kernel(GatherArgs A)
{
    __shared__ Lds L;
    const int lane = threadIdx.x;
    L.hist[lane] = 0;
    __syncthreads();
    constexpr uint32_t KPW = WAVE / G_LIGHT;     // light kernels per wave
    const uint32_t n_heavy = A.counts[0], n_light = A.counts[1];
    const uint32_t n_items = n_heavy + (n_light + KPW - 1) / KPW;
    uint64_t pairs = 0, cand = 0;
    for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
        if (item < n_heavy) {
            process<G_HEAVY, NRM, VCM>(A, L, (int64_t)A.heavy[item], true, pairs, cand);
        } else {
            const uint32_t li = (item - n_heavy) * KPW + (uint32_t)(lane / G_LIGHT);
            const bool act = li < n_light;
            const int64_t q = act ? (int64_t)A.light[li] : 0;
            process<G_LIGHT, NRM, VCM>(A, L, q, act, pairs, cand);
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

void launch_gather(const GatherArgs &a, bool nrm, bool vcm, hipStream_t s)
{
    if (a.H <= 0) return;
    const int grid = (int)cdiv(a.H, WAVE / G_LIGHT);
    if (nrm && vcm)
        gather_update_kernel<true, true><<<grid, WAVE, 0, s>>>(a);
    else if (nrm)
        gather_update_kernel<true, false><<<grid, WAVE, 0, s>>>(a);
    else if (vcm)
        gather_update_kernel<false, true><<<grid, WAVE, 0, s>>>(a);
    else
        gather_update_kernel<false, false><<<grid, WAVE, 0, s>>>(a);
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

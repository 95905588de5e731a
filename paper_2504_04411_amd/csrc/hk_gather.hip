// Fused gather, grouped compensated sums, ANOVA F-test and radius / estimate update for one set.
//
// Work decomposition: one wavefront (64 lanes) per tile of 64 kernels that are consecutive along
// the Morton curve; lane i owns kernel i of the tile for the whole iteration, so every sum is
// private to a lane and needs no atomics and no cross-lane reduction. The tile's photons are the
// grid cells overlapping the union of its disks: rows of cells (x fastest) are contiguous ranges of
// the sorted payload; the wave concatenates up to 64 rows, stages 64 photons at a time in LDS with
// coalesced loads, and every lane tests every staged photon against its own disk (LDS broadcast).
//
// Per kernel and pair inside the disk (Sec. 3.2, Sec. 5.1):
//   y = (<x - x*, u>, <x - x*, v>)             (Eq. map-function)
//   g = annulus (2 d2 >= r2) x sector (60 degree wedges from +u)
//   S_g += psi, Q_g += psi^2                  (compensated float32 pairs kept in LDS per lane)
//   flux sum += Phi (PPM) or w * beta (vertex merging, Eq. mis-weight with beta = 1)
// Epilogue per kernel: retained sums (Sec. 5.1), F in float64 (Eq. f-statistic) against the
// tabulated critical value for m = sum of J over the kept iterations, estimate update
// (Eq. progressive-VCM-estimator) with this iteration's radius, then Eq. radiusupdate.
#include <math.h>

#include "hk_fquant.h"
#include "hk_internal.h"
#include "hk_kernels.h"

namespace hk {

// Tile handled by workgroup b: workgroups are dealt to the 8 XCDs round-robin, so give each XCD a
// contiguous run of tiles (spatially close kernels share photons in that XCD's L2).
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int q = n >> 3, rem = n & 7;
    const int x = b & 7, j = b >> 3;
    return x * q + min(x, rem) + j;
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

template <bool NRM, bool VCM>
__global__ __launch_bounds__(TILE) void gather_update_kernel(GatherArgs A)
{
    __shared__ float4 slot[NG][TILE];          // per group and lane: S, comp S, Q, comp Q
    __shared__ float4 chA[CHUNK];              // photon x, y, z, luminance
    __shared__ float4 chN[NRM ? CHUNK : 1];    // photon normal
    __shared__ float4 chF[CHUNK];              // flux or throughput R, G, B; dVCM
    __shared__ float chM[VCM ? CHUNK : 1];     // dVM
    __shared__ uint32_t rstart[64];
    __shared__ uint32_t roff[64];
    __shared__ uint32_t lhist[RHIST_BINS];

    const int lane = threadIdx.x;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t q = (int64_t)tile * TILE + lane;
    const bool active = q < A.H;
    SetHeader *hdr = A.hdr;
    const int64_t ps = A.pstride;

    float x = 0.0f, y = 0.0f, z = 0.0f, r = 0.0f;
    float nx = 0.0f, ny = 0.0f, nz = 1.0f, ux = 1.0f, uy = 0.0f, uz = 0.0f, vx = 0.0f, vy = 1.0f, vz = 0.0f;
    if (active) {
        x = A.kp[0][q];
        y = A.kp[1][q];
        z = A.kp[2][q];
        r = A.r[q];
        ux = A.ku[0][q];
        uy = A.ku[1][q];
        uz = A.ku[2][q];
        vx = A.kv[0][q];
        vy = A.kv[1][q];
        vz = A.kv[2][q];
        if (NRM) {
            nx = A.kn[0][q];
            ny = A.kn[1][q];
            nz = A.kn[2][q];
        }
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
    for (int g = 0; g < NG; ++g)
        slot[g][lane] = active ? make_float4(A.sq[4 * g][q], A.sq[4 * g + 1][q], A.sq[4 * g + 2][q], A.sq[4 * g + 3][q])
                               : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    lhist[lane] = 0;

    float fR = 0.0f, cR = 0.0f, fG = 0.0f, cG = 0.0f, fB = 0.0f, cB = 0.0f;
    uint32_t cnt = 0;
    unsigned long long visited = 0;      // photons staged for this tile (wave-uniform)

    // union of the tile's disks, grown by a rounding margin, as a box of grid cells
    const float mg = active ? fmaf(r, 1e-4f, hdr->margin_abs) : 0.0f;
    const float p3[3] = {x, y, z};
    int c0[3], c1[3];
    bool any = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float lo = wave_min(active ? p3[a] - r - mg : INFINITY);
        const float hi = wave_max(active ? p3[a] + r + mg : -INFINITY);
        const float f0 = floorf((lo - hdr->dom_lo[a]) * hdr->cell_inv[a]);
        const float f1 = floorf((hi - hdr->dom_lo[a]) * hdr->cell_inv[a]);
        const float dm = (float)(hdr->dims[a] - 1);
        if (!(f0 <= f1)) any = false;
        c0[a] = (int)fminf(fmaxf(f0, 0.0f), dm);
        c1[a] = (int)fminf(fmaxf(f1, 0.0f), dm);
    }
    const int nyr = c1[1] - c0[1] + 1, nzr = c1[2] - c0[2] + 1;
    const int nrows = any ? nyr * nzr : 0;
    const int dimx = hdr->dims[0], dimy = hdr->dims[1];

    for (int rb = 0; rb < nrows; rb += 64) {
        const int row = rb + lane;
        uint32_t st = 0, len = 0;
        if (row < nrows) {
            const int cy = c0[1] + row % nyr, cz = c0[2] + row / nyr;
            const uint32_t base = ((uint32_t)cz * (uint32_t)dimy + (uint32_t)cy) * (uint32_t)dimx;
            st = A.cstart[base + (uint32_t)c0[0]];
            len = A.cstart[base + (uint32_t)c1[0] + 1u] - st;
        }
        const uint32_t inc = wave_incl_scan_u32(len);
        const uint32_t total = __shfl(inc, 63, 64);
        __syncthreads();
        rstart[lane] = st;
        roff[lane] = (row < nrows) ? inc - len : total;
        __syncthreads();
        for (uint32_t v0 = 0; v0 < total; v0 += CHUNK) {
            const uint32_t v = v0 + lane;
            if (v < total) {
                int j = 0;
#pragma unroll
                for (int step = 32; step > 0; step >>= 1)
                    if (roff[j + step] <= v) j += step;
                const int64_t p = (int64_t)rstart[j] + (v - roff[j]);
                chA[lane] = make_float4(A.pay[0 * ps + p], A.pay[1 * ps + p], A.pay[2 * ps + p], A.pay[9 * ps + p]);
                if (NRM) chN[lane] = make_float4(A.pay[3 * ps + p], A.pay[4 * ps + p], A.pay[5 * ps + p], 0.0f);
                chF[lane] = make_float4(A.pay[6 * ps + p], A.pay[7 * ps + p], A.pay[8 * ps + p],
                                        VCM ? A.pay[10 * ps + p] : 0.0f);
                if (VCM) chM[lane] = A.pay[11 * ps + p];
            }
            __syncthreads();
            const int nv = (int)min((uint32_t)CHUNK, total - v0);
            visited += (unsigned long long)nv;
            for (int k = 0; k < nv; ++k) {
                const float4 a = chA[k];
                const float dx = x - a.x, dy = y - a.y, dz = z - a.z;
                const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                bool in = d2 < r2;
                if (NRM) {
                    const float4 nn = chN[k];
                    const float c = fmaf(nz, nn.z, fmaf(ny, nn.y, nx * nn.x));
                    in = in && (c >= A.cos_min);
                }
                if (in) {
                    const float yu = fmaf(dz, uz, fmaf(dy, uy, dx * ux));
                    const float yv = fmaf(dz, vz, fmaf(dy, vy, dx * vx));
                    const int g = group_of(yu, yv, d2, r2);
                    const float4 f = chF[k];
                    float psi, wR, wG, wB;
                    if (VCM) {
                        const float wl = fmaf(chM[k], INV_PI_F, f.w * inv_eta);
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
                    float4 s = slot[g][lane];
                    kahan(s.x, s.y, psi);
                    kahan(s.z, s.w, psi * psi);
                    slot[g][lane] = s;
                    kahan(fR, cR, wR);
                    kahan(fG, cG, wG);
                    kahan(fB, cB, wB);
                    ++cnt;
                }
            }
            __syncthreads();
        }
    }

    if (active) {
        const uint32_t t_new = A.t[q] + 1u;
        const uint32_t seen = A.nseen[q] + cnt;
        const double m = A.mprefix[A.iter] - A.mprefix[A.iter - (int)t_new];
        double S[NG], Q[NG], tot = 0.0;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            const float4 s = slot[g][lane];
            S[g] = (double)s.x - (double)s.y;
            Q[g] = (double)s.z - (double)s.w;
            tot += S[g];
        }
        double ssb = 0.0, ssw = 0.0;
        const double mean = tot / NG;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            const double d = S[g] - mean;
            ssb += d * d;
            ssw += Q[g] - S[g] * S[g] / m;
        }
        ssb /= m;
        const double F = (ssb / (NG - 1)) / (ssw / (NG * (m - 1.0)));
        const double Fc = A.fctab[t_new];
        const bool valid = seen > 0u && ssw > 0.0 && m >= 2.0;
        const bool shrink = valid && (F > Fc);

        // this iteration's kernel estimate with its own radius
        const float denom = A.Jf * (PI_F * r2);
        float eR = (fR - cR) / denom, eG = (fG - cG) / denom, eB = (fB - cB) / denom;
        if (VCM) {
            eR = cbR * eR;
            eG = cbG * eG;
            eB = cbB * eB;
        }
        float tR = A.tau[0][q], tRc = A.tau[1][q], tG = A.tau[2][q], tGc = A.tau[3][q], tB = A.tau[4][q],
              tBc = A.tau[5][q];
        kahan(tR, tRc, eR);
        kahan(tG, tGc, eG);
        kahan(tB, tBc, eB);
        A.tau[0][q] = tR;
        A.tau[1][q] = tRc;
        A.tau[2][q] = tG;
        A.tau[3][q] = tGc;
        A.tau[4][q] = tB;
        A.tau[5][q] = tBc;

        const float rn = shrink ? fmaxf(A.k * r, A.lb) : r;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
            const float4 s = shrink ? make_float4(0.0f, 0.0f, 0.0f, 0.0f) : slot[g][lane];
            A.sq[4 * g][q] = s.x;
            A.sq[4 * g + 1][q] = s.y;
            A.sq[4 * g + 2][q] = s.z;
            A.sq[4 * g + 3][q] = s.w;
        }
        A.r[q] = rn;
        A.t[q] = shrink ? 0u : t_new;
        A.nseen[q] = shrink ? 0u : seen;
        A.cnt[q] = cnt;
        A.dec[q] = shrink ? 1u : 0u;
        A.F[q] = seen > 0u ? F : (double)NAN;
        A.Fc[q] = Fc;
        atomicAdd(&lhist[radius_bin(rn, A.r1)], 1u);
    }
    __syncthreads();
    if (lhist[lane]) atomicAdd(&hdr->rhist[lane], lhist[lane]);
    // tile totals for throughput accounting: in-disk pairs and lane x photon tests
    unsigned long long pairs = cnt;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) pairs += __shfl_xor(pairs, o, 64);
    const unsigned long long nact = (unsigned long long)__popcll(__ballot(active));
    if (lane == 0) {
        atomicAdd(&hdr->n_pairs, pairs);
        atomicAdd(&hdr->n_cand, visited * nact);
        if (blockIdx.x == 0) atomicAdd(&hdr->n_launch, 1ull);
    }
}

void launch_gather(const GatherArgs &a, bool nrm, bool vcm, hipStream_t s)
{
    if (a.ntiles <= 0) return;
    if (nrm && vcm)
        gather_update_kernel<true, true><<<a.ntiles, TILE, 0, s>>>(a);
    else if (nrm)
        gather_update_kernel<true, false><<<a.ntiles, TILE, 0, s>>>(a);
    else if (vcm)
        gather_update_kernel<false, true><<<a.ntiles, TILE, 0, s>>>(a);
    else
        gather_update_kernel<false, false><<<a.ntiles, TILE, 0, s>>>(a);
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

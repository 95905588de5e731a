// Uniform-grid build for the range search of one iteration (the "range search data structure" of
// Sec. 5.1) and the one-time set initialisation.
//
//   plan      picks the cell size from the radius distribution of the previous update
//   keys      cell index of every photon (x fastest), KEY_OUTSIDE outside the grid domain
//   sort      stable LSD radix sort of (key, photon index), 8-bit digits, per-chunk histograms, one
//             exclusive scan over them (digit-major), and a wave-ballot stable scatter
//   permute   the last sort pass writes the inverse permutation; a coalesced read / scattered write
//             of the photon payload into sorted order, one contiguous record per photon:
//             (position, luminance), (flux, dVCM) and, when read, (normal, dVM)
//   cstart    photons per cell (wave-aggregated atomics on the sorted keys), exclusive scan:
//             cstart[c] = first sorted position with key >= c, for c in [0, ncells]
#include <math.h>

#include "hk_internal.h"
#include "hk_kernels.h"

namespace hk {

// ------------------------------------------------------------------------------------------------
// scans
// ------------------------------------------------------------------------------------------------

// Length of a scan whose array is sized for a bound but whose live part is known on the device only
// (the cell counts of this iteration's plan): min(len, *dlen + extra), or len when dlen is NULL.
__device__ __forceinline__ int64_t live_len(int64_t len, const uint32_t *dlen, int extra)
{
    if (!dlen) return len;
    const int64_t l = (int64_t)*dlen + extra;
    return l < len ? l : len;
}

__global__ __launch_bounds__(256) void scan_reduce_kernel(const uint32_t *d, int64_t len, uint32_t *part,
                                                          const uint32_t *dlen, int extra)
{
    len = live_len(len, dlen, extra);
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    if (base >= len) {
        if (threadIdx.x == 0) part[blockIdx.x] = 0u;
        return;
    }
    // each thread sums its own run of SCAN_TILE / 256 counters (16-byte words when they are all
    // live and the array is 16-byte aligned)
    constexpr int PER = SCAN_TILE / 256;
    const int64_t first = base + (int64_t)threadIdx.x * PER;
    uint32_t s = 0;
    if (first + PER <= len && (reinterpret_cast<uintptr_t>(d) & 15u) == 0) {
#pragma unroll
        for (int i = 0; i < PER; i += 4) {
            const uint4 x = *reinterpret_cast<const uint4 *>(d + first + i);
            s += (x.x + x.y) + (x.z + x.w);
        }
    } else {
        for (int i = 0; i < PER; ++i) {
            const int64_t k = first + i;
            if (k < len) s += d[k];
        }
    }
    uint32_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void scan_down_kernel(uint32_t *d, int64_t len, const uint32_t *part,
                                                        const uint32_t *dlen, int extra)
{
    constexpr int PER = SCAN_TILE / 256;
    len = live_len(len, dlen, extra);
    if ((int64_t)blockIdx.x * SCAN_TILE >= len) return;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * PER;
    // a thread's PER counters as 16-byte words when they are all live and the array is 16-byte
    // aligned (a set's cell starts begin at any 4-byte offset of the batch's array)
    const bool vec = base + PER <= len && (reinterpret_cast<uintptr_t>(d) & 15u) == 0;
    uint32_t v[PER];
    uint32_t s = 0;
    if (vec) {
#pragma unroll
        for (int i = 0; i < PER; i += 4) {
            const uint4 x = *reinterpret_cast<const uint4 *>(d + base + i);
            v[i] = x.x;
            v[i + 1] = x.y;
            v[i + 2] = x.z;
            v[i + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int64_t k = base + i;
            v[i] = k < len ? d[k] : 0;
        }
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) s += v[i];
    // the block's offset: the partial sums of the blocks before it (each block adds them itself,
    // which saves a one-block launch between the two sweeps)
    uint32_t pre = 0;
    for (int i = threadIdx.x; i < (int)blockIdx.x; i += 256) pre += part[i];
    uint32_t off;
    block_excl_scan(pre, &off);
    uint32_t tot;
    uint32_t run = block_excl_scan(s, &tot) + off;
    if (vec) {
#pragma unroll
        for (int i = 0; i < PER; i += 4) {
            uint4 x;
            x.x = run;
            run += v[i];
            x.y = run;
            run += v[i + 1];
            x.z = run;
            run += v[i + 2];
            x.w = run;
            run += v[i + 3];
            *reinterpret_cast<uint4 *>(d + base + i) = x;
        }
    } else {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int64_t k = base + i;
            if (k < len) d[k] = run;
            run += v[i];
        }
    }
}

void excl_scan(uint32_t *d, int64_t len, uint32_t *part, hipStream_t s, const uint32_t *dlen, int extra)
{
    const int nparts = (int)cdiv(len, SCAN_TILE);
    scan_reduce_kernel<<<nparts, 256, 0, s>>>(d, len, part, dlen, extra);
    scan_down_kernel<<<nparts, 256, 0, s>>>(d, len, part, dlen, extra);
}

// ------------------------------------------------------------------------------------------------
// LSD radix sort of (key, value) pairs
// ------------------------------------------------------------------------------------------------

// Every wavefront of a radix block owns a chunk of RS_CHUNK consecutive keys (RS_ITEMS rounds of 64):
// segment seg = block * RS_WAVES + wave. Histograms, offsets and the scatter are per segment, so the
// scatter's waves never wait for each other.
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int RS_CHUNK = 64 * RS_ITEMS;
static_assert(RS_TILE == RS_WAVES * RS_CHUNK, "a radix block is its waves' chunks");

// Workgroups are dealt to the 8 XCDs round-robin. A radix launch has 8 * per workgroups, and
// workgroup b takes block (b mod 8) * per + b / 8: each XCD walks one contiguous range of blocks, so
// the short runs that neighbouring chunks write into each digit's range (and their histogram
// columns) fill whole cache lines in one L2 instead of partial lines in several. Returns -1 for
// the padding workgroups past the last block.
__host__ __device__ constexpr int rs_per_xcd(int nblk) { return (nblk + 7) / 8; }
__device__ __forceinline__ int rs_block(int nblk)
{
    const int b = (int)blockIdx.x, blk = (b & 7) * rs_per_xcd(nblk) + (b >> 3);
    return blk < nblk ? blk : -1;
}

// Digit counts of every segment of the block: hist[d * nseg + seg]. The chunk's keys are loaded
// together (RS_ITEMS loads in flight per lane), then counted in the wave's own LDS histogram.
__device__ __forceinline__ void rs_count_store(uint32_t (&cnt)[RS_WAVES][256], uint32_t *hist, int nseg, int blk)
{
    __syncthreads();
    const int seg0 = blk * RS_WAVES;
    for (int i = threadIdx.x; i < RS_WAVES * 256; i += RS_THREADS) {
        const int w = i & (RS_WAVES - 1), d = i / RS_WAVES;
        if (seg0 + w < nseg) hist[(int64_t)d * nseg + seg0 + w] = cnt[w][d];
    }
}

__global__ __launch_bounds__(RS_THREADS) void rs_hist_kernel(const uint32_t *keys, int64_t n, int shift,
                                                             uint32_t *hist, int nseg, int nblk)
{
    __shared__ uint32_t cnt[RS_WAVES][256];
    const int blk = rs_block(nblk);
    if (blk < 0) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < RS_WAVES * 256; i += RS_THREADS) (&cnt[0][0])[i] = 0u;
    __syncthreads();
    const int64_t base = ((int64_t)blk * RS_WAVES + w) * RS_CHUNK + lane;
    uint32_t k[RS_ITEMS];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) k[i] = base + 64 * i < n ? keys[base + 64 * i] : 0u;
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i)
        if (base + 64 * i < n) atomicAdd(&cnt[w][(k[i] >> shift) & 255u], 1u);
    rs_count_store(cnt, hist, nseg, blk);
}

// Waves per scatter workgroup. One: a workgroup's 10 KB of LDS fits beside a CU's full load of
// gather wavefronts (12 x 12.5 KB of the 160 KB), so a set's sort can progress while another phase's
// gather runs; a four-wave workgroup's 40 KB waits for the gather to drain.
constexpr int RS_SCATTER_WAVES = 1;

// Stable scatter, one wavefront per segment and no barrier between the block's waves. The counts
// hist[d * nseg + seg], scanned as one array (digit-major), give each segment's first position for
// digit d: all keys of smaller digits, then those of digit d in earlier segments. The wave first
// sorts its chunk locally: the chunk's digit counts and their scan give each digit's local start,
// the chunk is visited in rounds of 64 consecutive keys, a key's rank among the round's equal
// digits comes from eight ballots, and the first lane of each digit advances the digit's running
// local position (a wave's LDS accesses are performed in order, so the next round reads the
// advanced value). Keys and values are staged in LDS in that order and then written out in it:
// neighbouring lanes mostly hold the same digit, so their global positions are neighbours too.
// With `inv` (the last pass), the inverse permutation is written instead of the sorted values:
// inv[source index] = sorted position.
template <int SW>
__global__ __launch_bounds__(64 * SW) void rs_scatter_kernel(const uint32_t *kin, const uint32_t *vin,
                                                             uint32_t *kout, uint32_t *vout, int64_t n, int shift,
                                                             const uint32_t *offs, int nseg, uint32_t *inv)
{
    __shared__ uint32_t gbase[SW][256];             // global start of each digit minus its local start
    __shared__ uint32_t lrow[SW][256];              // counts, then the running local position per digit
    __shared__ uint32_t sk[SW][RS_CHUNK], sv[SW][RS_CHUNK];
    const int blk = rs_block((nseg + SW - 1) / SW);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int seg = blk * SW + w;
    if (blk < 0 || seg >= nseg) return;
    const int64_t base = (int64_t)seg * RS_CHUNK + lane;
    uint32_t k[RS_ITEMS], v[RS_ITEMS];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int64_t q = base + 64 * i;
        k[i] = q < n ? kin[q] : 0u;
        v[i] = vin ? (q < n ? vin[q] : 0u) : (uint32_t)q;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) lrow[w][4 * lane + j] = 0u;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i)
        if (base + 64 * i < n) atomicAdd(&lrow[w][(k[i] >> shift) & 255u], 1u);
    __builtin_amdgcn_wave_barrier();
    uint32_t c[4], sum = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        c[j] = lrow[w][4 * lane + j];
        sum += c[j];
    }
    uint32_t ex = wave_incl_scan(sum) - sum;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int d = 4 * lane + j;
        lrow[w][d] = ex;
        gbase[w][d] = offs[(int64_t)d * nseg + seg] - ex;
        ex += c[j];
    }
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const bool valid = base + 64 * i < n;
        const uint32_t d = (k[i] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = __popcll(peers & lt);
        const uint32_t pos = lrow[w][d] + rank;
        __builtin_amdgcn_wave_barrier();
        if (valid) {
            sk[w][pos] = k[i];
            sv[w][pos] = v[i];
            if (rank == 0) lrow[w][d] = pos + (uint32_t)__popcll(peers);
        }
        __builtin_amdgcn_wave_barrier();
    }
    const int64_t left = n - (int64_t)seg * RS_CHUNK;
    const int nvalid = left < RS_CHUNK ? (int)left : RS_CHUNK;
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int p = 64 * i + lane;
        if (p < nvalid) {
            const uint32_t key = sk[w][p], val = sv[w][p];
            const uint32_t pos = gbase[w][(key >> shift) & 255u] + (uint32_t)p;
            kout[pos] = key;
            if (inv)
                inv[val] = pos;
            else
                vout[pos] = val;
        }
    }
}

// Sorts n pairs whose keys use `bits` low bits. Values start as the identity permutation. Returns
// in *kres whichever buffer holds the sorted keys and in *vres the one holding the sorted values
// (sorted position -> source index), or with `inverse` the inverse permutation (source index ->
// sorted position), which the last pass then writes instead.
void radix_sort(uint32_t *kA, uint32_t *vA, uint32_t *kB, uint32_t *vB, int64_t n, int bits, uint32_t *hist,
                uint32_t *part, hipStream_t s, uint32_t **kres, uint32_t **vres, bool inverse, bool first_hist_done)
{
    const int nblk = (int)cdiv(n, RS_TILE);
    const int nseg = (int)cdiv(n, RS_CHUNK);
    const int grid = 8 * rs_per_xcd(nblk);
    uint32_t *ki = kA, *vi = nullptr, *ko = kB, *vo = vB;
    uint32_t *vspare = vA;
    for (int shift = 0; shift < bits; shift += 8) {
        const bool last = shift + 8 >= bits;
        if (shift > 0 || !first_hist_done)
            rs_hist_kernel<<<grid, RS_THREADS, 0, s>>>(ki, n, shift, hist, nseg, nblk);
        excl_scan(hist, (int64_t)256 * nseg, part, s, nullptr, 0);
        rs_scatter_kernel<RS_SCATTER_WAVES><<<8 * rs_per_xcd((int)cdiv(nseg, RS_SCATTER_WAVES)),
                                              64 * RS_SCATTER_WAVES, 0, s>>>(ki, vi, ko, vo, n, shift, hist, nseg,
                                                                             (last && inverse) ? vo : nullptr);
        uint32_t *kt = ki;
        ki = ko;
        ko = kt;
        uint32_t *vt = vi ? vi : vspare;
        vi = vo;
        vo = vt;
    }
    *kres = ki;
    *vres = vi;
}

// ------------------------------------------------------------------------------------------------
// per-iteration grid
// ------------------------------------------------------------------------------------------------

// Cells are CELL_XSUB times narrower along x than along y and z. A stencil row runs along x and is
// clipped to whole cells, so finer x cells cut the candidates a row carries beyond its chord of the
// disk (about 2.0 -> 1.6 candidates per in-disk photon for a disk in a plane that contains the rows,
// cell 0.7 r, with four; eight take the gather another 1.5-2% lower) without adding rows; the cost
// is CELL_XSUB times more cell starts to zero and scan.
constexpr float CELL_XSUB = 8.0f;

// One wavefront: advance the set's iteration counter, append J to the prefix sums, choose the cell
// size from the radius histogram (y and z; x a CELL_XSUB-th of it). The quantile's bin is the
// largest b whose count of radii in bins >= b reaches the target: lane b holds bin b, the counts
// from the top come from a suffix scan. Everything that changes between iterations lives in the
// state, so a captured graph can replay the iteration.
static_assert(RHIST_BINS == WAVE, "one lane per radius bin");
__device__ void plan_set(SetHeader *hdr, double *mprefix, double J, float cell_scale, float quantile,
                         uint32_t max_cells)
{
    const int b = (int)threadIdx.x;
    uint64_t above = hdr->rhist[b];
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const uint64_t v = __shfl_down(above, o, WAVE);
        if (b + o < WAVE) above += v;
    }
    const double target = (double)quantile * hdr->H;
    const uint64_t reach = __ballot((double)above >= target);
    const int bq = reach ? 63 - __clzll((long long)reach) : 0;
    hdr->rhist[b] = 0;
    if (b != 0) return;
    const int iter = hdr->iter + 1;
    hdr->iter = iter;
    hdr->Jf = (float)J;
    hdr->n_launch += 1ull;
    mprefix[iter] = mprefix[iter - 1] + J;
    float cell = cell_scale * hdr->r1 * exp2f(-0.25f * (float)bq);
    float ext[3];
    int flat[3];
    float emax = 0.0f;
    for (int a = 0; a < 3; ++a) {
        ext[a] = hdr->dom_hi[a] - hdr->dom_lo[a];
        emax = fmaxf(emax, ext[a]);
    }
    for (int a = 0; a < 3; ++a) flat[a] = hdr->kflat[a];
    if (!(cell > 0.0f)) cell = emax;
    int dims[3];
    for (int guard = 0; guard < 200; ++guard) {
        double tot = 1.0;
        for (int a = 0; a < 3; ++a) {
            float q = floorf(ext[a] * (a == 0 ? CELL_XSUB : 1.0f) / cell);
            int d = (q < 1.0f || flat[a]) ? 1 : (q > 65535.0f ? 65535 : (int)q);
            dims[a] = d;
            tot *= d;
        }
        if (tot <= (double)max_cells) break;
        cell *= 1.25f;
    }
    for (int a = 0; a < 3; ++a) {
        hdr->dims[a] = dims[a];
        hdr->cell_inv[a] = (float)dims[a] / ext[a];
    }
    hdr->ncells = (uint32_t)dims[0] * (uint32_t)dims[1] * (uint32_t)dims[2];
    hdr->cell = cell;
}

// One wavefront per set of a batch.
struct PlanBatch {
    const SetDesc *desc;
    float cell_scale, quantile;
    double J[MAX_BATCH];
};

__global__ __launch_bounds__(WAVE) void plan_batch_kernel(PlanBatch P)
{
    const SetDesc D = P.desc[blockIdx.x];
    plan_set(reinterpret_cast<SetHeader *>(D.state + D.hdr), reinterpret_cast<double *>(D.state + D.mprefix),
             P.J[blockIdx.x], P.cell_scale, P.quantile, D.max_cells);
}

// One thread: a grid of fixed cell size `cell` (grown until the cell count fits max_cells) over the
// set's domain, without advancing the iteration (used to count light vertices around the kernels
// outside an iteration).
__global__ void plan_fixed_kernel(SetHeader *hdr, float cell, uint32_t max_cells)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float ext[3], emax = 0.0f;
    for (int a = 0; a < 3; ++a) {
        ext[a] = hdr->dom_hi[a] - hdr->dom_lo[a];
        emax = fmaxf(emax, ext[a]);
    }
    if (!(cell > 0.0f)) cell = emax;
    int dims[3];
    for (int guard = 0; guard < 200; ++guard) {
        double tot = 1.0;
        for (int a = 0; a < 3; ++a) {
            float q = floorf(ext[a] / cell);
            int d = (q < 1.0f || hdr->kflat[a]) ? 1 : (q > 65535.0f ? 65535 : (int)q);
            dims[a] = d;
            tot *= d;
        }
        if (tot <= (double)max_cells) break;
        cell *= 1.25f;
    }
    for (int a = 0; a < 3; ++a) {
        hdr->dims[a] = dims[a];
        hdr->cell_inv[a] = (float)dims[a] / ext[a];
    }
    hdr->ncells = (uint32_t)dims[0] * (uint32_t)dims[1] * (uint32_t)dims[2];
    hdr->cell = cell;
}

void launch_plan_fixed(SetHeader *hdr, float cell, uint32_t max_cells, hipStream_t s)
{
    plan_fixed_kernel<<<1, 64, 0, s>>>(hdr, cell, max_cells);
}

// The plan's grid: domain corner, cells per unit length and cell counts per axis.
struct GridPlan {
    float lo[3], inv[3];
    int dims[3];
};

__device__ __forceinline__ GridPlan grid_plan(const SetHeader *hdr)
{
    GridPlan g;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = hdr->dom_lo[a];
        g.inv[a] = hdr->cell_inv[a];
        g.dims[a] = hdr->dims[a];
    }
    return g;
}

__device__ __forceinline__ uint32_t cell_key(const GridPlan &g, float x, float y, float z)
{
    const float p[3] = {x, y, z};
    uint32_t c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float f = floorf((p[a] - g.lo[a]) * g.inv[a]);
        if (!(f >= 0.0f && f < (float)g.dims[a])) return KEY_OUTSIDE;
        c[a] = (uint32_t)f;
    }
    return (c[2] * (uint32_t)g.dims[1] + c[1]) * (uint32_t)g.dims[0] + c[0];
}

// Cell keys of a radix block's photons together with their segments' histograms of the low 8 bits
// (the first sort pass's histogram, laid out as rs_hist_kernel writes it). A lane loads the positions
// of its RS_ITEMS keys together.
__global__ __launch_bounds__(RS_THREADS) void keys_hist_kernel(const SetHeader *hdr, const float *px,
                                                               const float *py, const float *pz, int64_t n,
                                                               uint32_t *keys, uint32_t *hist, int nseg, int nblk)
{
    __shared__ uint32_t cnt[RS_WAVES][256];
    const int blk = rs_block(nblk);
    if (blk < 0) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < RS_WAVES * 256; i += RS_THREADS) (&cnt[0][0])[i] = 0u;
    const GridPlan gp = grid_plan(hdr);
    __syncthreads();
    const int64_t base = ((int64_t)blk * RS_WAVES + w) * RS_CHUNK + lane;
    float x[RS_ITEMS], y[RS_ITEMS], z[RS_ITEMS];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int64_t q = base + 64 * i;
        const bool in = q < n;
        x[i] = in ? px[q] : 0.0f;
        y[i] = in ? py[q] : 0.0f;
        z[i] = in ? pz[q] : 0.0f;
    }
#pragma unroll
    for (int i = 0; i < RS_ITEMS; ++i) {
        const int64_t q = base + 64 * i;
        if (q < n) {
            const uint32_t key = cell_key(gp, x[i], y[i], z[i]);
            keys[q] = key;
            atomicAdd(&cnt[w][key & 255u], 1u);
        }
    }
    rs_count_store(cnt, hist, nseg, blk);
}

// inv[original index] = sorted position
// Reads the input photons in their own order (coalesced) and writes each one's record, `rec` float4s,
// at its sorted position. The record is written by neighbouring lanes, one float4 each (two lanes
// per photon for two-float4 records, four for three), so one store instruction of a wavefront writes
// 32 or 16 whole records (as many contiguous regions) rather than one float4 of 64 records at 64
// scattered places.
__global__ __launch_bounds__(256) void permute_kernel(PhotonSrc src, int64_t n, const uint32_t *inv, float4 *recs,
                                                      int rec)
{
    const int lg = rec == 2 ? 1 : 2;            // log2 of the lanes per photon
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j = t >> lg;                  // the photon
    const int part = (int)(t & ((1 << lg) - 1));   // which float4 of its record
    if (j >= n || part >= rec) return;
    const uint32_t q = inv[j];
    float4 v;
    if (part == 0) {
        const float R = src.flux[0][j], G = src.flux[1][j], B = src.flux[2][j];
        v = make_float4(src.pos[0][j], src.pos[1][j], src.pos[2][j], luminance(R, G, B));
    } else if (part == 1) {
        v = make_float4(src.flux[0][j], src.flux[1][j], src.flux[2][j], src.mis[0] ? src.mis[0][j] : 0.0f);
    } else {
        // the (normal, dVM) entry exists only where a normal test or vertex merging reads it
        const float dvm = src.mis[0] ? src.mis[2][j] : 0.0f;
        v = src.nrm[0] ? make_float4(src.nrm[0][j], src.nrm[1][j], src.nrm[2][j], dvm)
                       : make_float4(0.0f, 0.0f, 1.0f, dvm);
    }
    recs[(int64_t)q * rec + part] = v;
}

// Four counters per thread: one 16-byte store when all four are live and the array is 16-byte
// aligned, else one store each.
constexpr int ZERO_PER = 4;
__global__ __launch_bounds__(256) void zero_kernel(uint32_t *p, int64_t n, const uint32_t *dlen, int extra)
{
    const int64_t i = ((int64_t)blockIdx.x * 256 + threadIdx.x) * ZERO_PER;
    const int64_t len = live_len(n, dlen, extra);
    if (i + ZERO_PER <= len && (reinterpret_cast<uintptr_t>(p) & 15u) == 0) {
        *reinterpret_cast<uint4 *>(p + i) = make_uint4(0u, 0u, 0u, 0u);
    } else {
        for (int k = 0; k < ZERO_PER; ++k)
            if (i + k < len) p[i + k] = 0u;
    }
}

// Photons per cell from the sorted keys: the first lane of every run of equal keys inside a
// wavefront adds the run length (a handful of atomics per wavefront).
__global__ __launch_bounds__(256) void cell_count_kernel(const SetHeader *hdr, const uint32_t *skeys, int64_t n,
                                                         uint32_t *cnt)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const uint32_t key = q < n ? skeys[q] : KEY_OUTSIDE;
    const uint32_t prev = __shfl_up(key, 1, 64);
    const bool head = (lane == 0) || (key != prev);
    const uint64_t heads = __ballot(head);
    if (head && q < n && key < hdr->ncells) {
        const uint64_t later = (lane == 63) ? 0ull : (heads >> (lane + 1));
        const int next = later ? lane + 1 + __builtin_ctzll(later) : 64;
        atomicAdd(&cnt[key], (uint32_t)(next - lane));
    }
}

void launch_zero(uint32_t *p, int64_t n, hipStream_t s)
{
    if (n > 0) zero_kernel<<<(int)cdiv(n, 256 * ZERO_PER), 256, 0, s>>>(p, n, nullptr, 0);
}

void build_grid(const GridLaunch &g, hipStream_t s)
{
    const int64_t n = g.n;
    // counts of every cell of this iteration's plan, then their scan: the arrays are sized for the
    // workspace bound, the plan's cell count (on the device) limits the work
    const int64_t nc = (int64_t)g.ncells_bound + 1;
    zero_kernel<<<(int)cdiv(nc, 256 * ZERO_PER), 256, 0, s>>>(g.cstart, nc, &g.hdr->ncells, 1);
    if (n > 0) {
        const int nb = (int)cdiv(n, 256);
        const int nblk = (int)cdiv(n, RS_TILE);
        keys_hist_kernel<<<8 * rs_per_xcd(nblk), RS_THREADS, 0, s>>>(g.hdr, g.src.pos[0], g.src.pos[1],
                                                                      g.src.pos[2], n, g.keyA, g.hist,
                                                                      (int)cdiv(n, RS_CHUNK), nblk);
        uint32_t *ks, *inv;
        radix_sort(g.keyA, g.valA, g.keyB, g.valB, n, 24, g.hist, g.part, s, &ks, &inv, true, true);
        permute_kernel<<<(int)cdiv((g.rec == 2 ? 2 : 4) * n, 256), 256, 0, s>>>(g.src, n, inv,
                                                                            g.pay + g.pay_off * g.rec, g.rec);
        cell_count_kernel<<<nb, 256, 0, s>>>(g.hdr, ks, n, g.cstart);
    }
    excl_scan(g.cstart, nc, g.part3, s, &g.hdr->ncells, 1);
}

// ------------------------------------------------------------------------------------------------
// set initialisation
// ------------------------------------------------------------------------------------------------

// One block: bounding box of the kernels, largest initial radius, grid domain and header fields.
__global__ __launch_bounds__(1024) void bbox_kernel(SetHeader *hdr, double *mprefix, int max_iters,
                                                    const float *px, const float *py, const float *pz,
                                                    const float *r_init, int64_t n, float r1, float r_floor,
                                                    int has_nrm, int vcm)
{
    __shared__ float red[7][16];
    __shared__ uint32_t nbad[16];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, rm = r1;
    uint32_t bad = 0;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
        const float p[3] = {px[i], py[i], pz[i]};
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], p[a]);
            hi[a] = fmaxf(hi[a], p[a]);
        }
        if (r_init) {
            const float r = r_init[i];
            // a radius below the first lower bound could grow at its first shrink (Eq. radiusupdate)
            bad += (isfinite(r) && r > 0.0f && r >= r_floor) ? 0u : 1u;
            rm = fmaxf(rm, r);
        }
    }
    float v[7] = {lo[0], lo[1], lo[2], -hi[0], -hi[1], -hi[2], -rm};
    for (int k = 0; k < 7; ++k)
        for (int o = 32; o > 0; o >>= 1) v[k] = fminf(v[k], __shfl_xor(v[k], o, 64));
    for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        for (int k = 0; k < 7; ++k) red[k][w] = v[k];
        nbad[w] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < 7; ++k) {
            float m = red[k][0];
            for (int i = 1; i < 16; ++i) m = fminf(m, red[k][i]);
            v[k] = m;
        }
        uint32_t nb = 0;
        for (int i = 0; i < 16; ++i) nb += nbad[i];
        hdr->n_bad_r = nb;
        float kl[3] = {v[0], v[1], v[2]}, kh[3] = {-v[3], -v[4], -v[5]};
        const float rmax = -v[6];
        float scale = 0.0f;
        for (int a = 0; a < 3; ++a) scale = fmaxf(scale, fmaxf(fabsf(kl[a]), fabsf(kh[a])));
        scale += rmax;
        const float margin = 4e-6f * fmaxf(scale, 1e-30f);
        float ext = 0.0f;
        for (int a = 0; a < 3; ++a) ext = fmaxf(ext, kh[a] - kl[a]);
        for (int a = 0; a < 3; ++a) {
            const float grow = rmax * 1.001f + 4.0f * margin;
            hdr->dom_lo[a] = kl[a] - grow;
            hdr->dom_hi[a] = kh[a] + grow;
            hdr->kb_lo[a] = kl[a];
            hdr->kb_hi[a] = kh[a];
            hdr->kflat[a] = (kh[a] - kl[a]) <= 1e-6f * ext ? 1 : 0;
        }
        hdr->margin_abs = margin;
        hdr->r1 = r1;
        hdr->rmax0 = rmax;
        hdr->H = (int32_t)n;
        hdr->has_nrm = has_nrm;
        hdr->vcm = vcm;
        hdr->max_iters = max_iters;
        for (int b = 0; b < RHIST_BINS; ++b) hdr->rhist[b] = 0;
        hdr->n_launch = 0;
        hdr->n_pairs = 0;
        hdr->n_cand = 0;
        hdr->iter = 0;
        hdr->Jf = 0.0f;
    }
    for (int i = threadIdx.x; i < max_iters + 2; i += 1024) mprefix[i] = 0.0;
}

__device__ __forceinline__ uint32_t spread10(uint32_t x)
{
    x &= 0x3FFu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__global__ __launch_bounds__(256) void morton_kernel(const SetHeader *hdr, const float *px, const float *py,
                                                     const float *pz, int64_t n, uint32_t *keys)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float p[3] = {px[i], py[i], pz[i]};
    uint32_t c[3];
    for (int a = 0; a < 3; ++a) {
        const float e = hdr->kb_hi[a] - hdr->kb_lo[a];
        float f = e > 0.0f ? (p[a] - hdr->kb_lo[a]) / e * 1023.0f : 0.0f;
        f = fminf(fmaxf(f, 0.0f), 1023.0f);
        c[a] = (uint32_t)f;
    }
    keys[i] = spread10(c[0]) | (spread10(c[1]) << 1) | (spread10(c[2]) << 2);
}

// One hit point s of the Morton-ordered set: copy, tangent frame, cleared statistics; its radius
// goes to the block's histogram.
__device__ void init_one(const KernelSrc &src, const StateView &st, const uint32_t *perm, int64_t s, float r1,
                         uint32_t *hist)
{
    const uint32_t j = perm[s];
    for (int a = 0; a < 3; ++a) st.pos[a][s] = src.pos[a][j];
    float nv[3] = {0.0f, 0.0f, 1.0f};
    if (src.nrm[0])
        for (int a = 0; a < 3; ++a) nv[a] = src.nrm[a][j];
    float u[3], v[3];
    onb(nv[0], nv[1], nv[2], u, v);
    for (int a = 0; a < 3; ++a) {
        st.nrm[a][s] = nv[a];
        st.u[a][s] = u[a];
        st.v[a][s] = v[a];
    }
    const float r = src.r_init ? src.r_init[j] : r1;
    st.r[s] = r;
    st.t[s] = 0;
    st.nseen[s] = 0;
    st.orig[s] = j;
    st.cnt[s] = 0;
    st.dec[s] = 0;
    st.cand[s] = 0;
    for (int i = 0; i < NG * st.nch; ++i) st.sq2[(size_t)s * (NG * st.nch) + i] = make_double2(0.0, 0.0);
    for (int i = 0; i < 6; ++i) st.tau0[(size_t)i * st.astride + s] = 0.0f;
    st.F[s] = NAN;
    st.Fc[s] = NAN;
    if (src.cam_beta[0]) {
        for (int a = 0; a < 3; ++a) st.cb[a][s] = src.cam_beta[a][j];
        st.cdvcm[s] = src.cam_mis[0][j];
        st.cdvm[s] = src.cam_mis[2][j];
    }
    atomicAdd(&hist[radius_bin(r, r1)], 1u);
}

__global__ __launch_bounds__(256) void init_state_kernel(KernelSrc src, StateView st, const uint32_t *perm,
                                                         int64_t n, float r1)
{
    __shared__ uint32_t hist[RHIST_BINS];
    if (threadIdx.x < RHIST_BINS) hist[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s < n) init_one(src, st, perm, s, r1, hist);
    __syncthreads();
    if (threadIdx.x < RHIST_BINS && hist[threadIdx.x]) atomicAdd(&st.hdr->rhist[threadIdx.x], hist[threadIdx.x]);
}

void init_set(const InitLaunch &g, hipStream_t s)
{
    const int64_t n = g.n;
    bbox_kernel<<<1, 1024, 0, s>>>(g.st.hdr, g.st.mprefix, g.max_iters, g.src.pos[0], g.src.pos[1], g.src.pos[2],
                                   g.src.r_init, n, g.r1, g.r_floor, g.src.nrm[0] != nullptr, g.vcm);
    const int nb = (int)cdiv(n, 256);
    morton_kernel<<<nb, 256, 0, s>>>(g.st.hdr, g.src.pos[0], g.src.pos[1], g.src.pos[2], n, g.keyA);
    uint32_t *ks, *vs;
    radix_sort(g.keyA, g.valA, g.keyB, g.valB, n, 30, g.hist, g.part, s, &ks, &vs, false, false);
    init_state_kernel<<<nb, 256, 0, s>>>(g.src, g.st, vs, n, g.r1);
}

}  // namespace hk

namespace hk {
void launch_plan_batch(const SetDesc *desc, int nb, const double *J, float cell_scale, float quantile,
                       hipStream_t s)
{
    PlanBatch P{};
    P.desc = desc;
    P.cell_scale = cell_scale;
    P.quantile = quantile;
    for (int k = 0; k < nb && k < MAX_BATCH; ++k) P.J[k] = J[k];
    plan_batch_kernel<<<nb, WAVE, 0, s>>>(P);
}
// Small host tables (the set records of a batch, the radius lower bounds) travel to the device in
// kernel arguments, UPLOAD_WORDS words per launch: the copy is ordered on the stream, needs no host
// buffer that outlives the call, and is an ordinary kernel node when the sequence is captured.
constexpr int UPLOAD_WORDS = 128;
struct UploadChunk {
    uint32_t w[UPLOAD_WORDS];
};

__global__ __launch_bounds__(UPLOAD_WORDS) void upload_kernel(uint32_t *dst, UploadChunk c, int n)
{
    if ((int)threadIdx.x < n) dst[threadIdx.x] = c.w[threadIdx.x];
}

void launch_upload(void *dst, const void *src, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 4;
    const uint32_t *w = static_cast<const uint32_t *>(src);
    uint32_t *d = static_cast<uint32_t *>(dst);
    for (size_t i = 0; i < n; i += UPLOAD_WORDS) {
        UploadChunk c{};
        const int k = (int)((n - i < (size_t)UPLOAD_WORDS) ? n - i : (size_t)UPLOAD_WORDS);
        for (int j = 0; j < k; ++j) c.w[j] = w[i + j];
        upload_kernel<<<1, UPLOAD_WORDS, 0, s>>>(d + i, c, k);
    }
}

}  // namespace hk

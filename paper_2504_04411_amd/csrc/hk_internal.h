// Internal definitions of libhk: per-set state layout, device helpers, kernel launch declarations.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "hk.h"

namespace hk {

constexpr int NG = 12;              // 2 annuli x 6 sectors (Sec. 6.1.1)
constexpr int NSQ = 4 * NG;         // per group: S and Q as float64 (four float-sized slots)
constexpr int RHIST_BINS = 64;      // radius histogram: bin = floor(-4 log2(r / r1))
constexpr uint32_t KEY_OUTSIDE = 0xFFFFFFu;   // cell key of a photon outside the grid domain
constexpr uint32_t MAX_CELLS = 0xFFFFF0u;     // keys fit 24 bits: three 8-bit radix passes
constexpr int WAVE = 64;            // wavefront width of gfx950
constexpr int MAX_BATCH = 64;       // sets gathered by one launch (6 bits of a work-list entry)
constexpr uint32_t Q_BITS = 26;     // kernel index bits of a work-list entry
constexpr float PI_F = 3.14159265358979323846f;
constexpr float INV_PI_F = 0.31830988618379067f;

// Set header at the start of each set's state buffer (device resident).
struct SetHeader {
    int32_t H;
    int32_t has_nrm;
    int32_t vcm;
    int32_t max_iters;
    float dom_lo[3];         // grid domain: kernel bounding box grown by r1 and a rounding margin
    float dom_hi[3];
    float margin_abs;        // absolute rounding margin for cell ranges
    float r1;
    float rmax0;             // largest initial radius
    float kb_lo[3];          // bounding box of the kernels
    float kb_hi[3];
    int32_t kflat[3];        // 1 where every kernel has the same coordinate (one cell on that axis)
    uint32_t rhist[RHIST_BINS];   // radii histogram written by the update, read by the next plan
    // plan of the current iteration (written on the device by the plan kernel)
    float cell_inv[3];       // cells per unit length per axis
    int32_t dims[3];
    uint32_t ncells;
    float cell;
    int32_t iter;            // iterations started (the plan kernel advances it)
    float Jf;                // J_emitted of the current iteration
    uint32_t n_bad_r;        // caller radii (r_init) that are not finite or below r_min, counted at set-up
    int32_t pad;
    // running totals since hk_set_kernels (gather launches, in-disk pairs, lane x photon tests)
    unsigned long long n_launch;
    unsigned long long n_pairs;
    unsigned long long n_cand;
};

// Per-kernel arrays of a set's state, by slot: every slot is `stride` bytes (256-byte aligned, one
// float or uint32 per kernel); float64 arrays take two slots.
// The group sums come last: NSQ slots per test channel (1, or 3 with one test per RGB channel).
enum Slot : int {
    SL_POS = 0, SL_NRM = 3, SL_U = 6, SL_V = 9, SL_R = 12, SL_T = 13, SL_NSEEN = 14, SL_ORIG = 15, SL_CNT = 16,
    SL_DEC = 17, SL_TAU = 18, SL_F = SL_TAU + 6, SL_FC = SL_F + 2, SL_CB = SL_FC + 2, SL_CDVCM = SL_CB + 3,
    SL_CDVM = SL_CDVCM + 1, SL_CAND = SL_CDVM + 1, SL_SQ = SL_CAND + 1
};

constexpr int slot_count(int nch) { return SL_SQ + NSQ * nch; }

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Offsets (bytes) in a set's state buffer.
struct Layout {
    int64_t H = 0;
    int max_iters = 0;
    int nch = 1;                    // test channels
    size_t hdr = 0, mprefix = 0, fctab = 0, lbtab = 0, arr = 0, stride = 0, total = 0;
    size_t slot(int k) const { return arr + (size_t)k * stride; }
};

inline Layout make_layout(int64_t H, int max_iters, int nch)
{
    Layout L;
    L.H = H;
    L.max_iters = max_iters;
    L.nch = nch;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    L.hdr = take(sizeof(SetHeader));
    L.mprefix = take(sizeof(double) * (max_iters + 2));
    L.fctab = take(sizeof(double) * (max_iters + 2));
    L.lbtab = take(sizeof(float) * (max_iters + 2));
    L.stride = align256(sizeof(float) * (size_t)H);
    L.arr = off;
    L.total = L.arr + (size_t)slot_count(nch) * L.stride;
    return L;
}

// Device view of one set's state (raw pointers into the caller's buffer).
struct StateView {
    SetHeader *hdr;
    double *mprefix;     // mprefix[i] = sum of J over iterations 1..i
    double *fctab;       // fctab[t] = critical value for t kept iterations
    float *lbtab;        // lbtab[i] = r_min sqrt(i^(alpha-1)), float32
    float *pos[3], *nrm[3], *u[3], *v[3];
    float *r;
    uint32_t *t, *nseen, *orig, *cnt, *dec;
    uint32_t *cand;      // candidate tests of the last iteration (the next work list's cost estimate)
    float *sq0;          // group sums: NSQ * nch slots holding, per hit point s, NG * nch double2s
    double2 *sq2;        // (S, Q) at sq2[s * NG * nch + column], column = channel * NG + group
    int nch;             // test channels
    float *tau0;         // estimate: array c at tau0 + c * astride
    uint32_t astride;    // floats between slots
    double *F, *Fc;
    float *cb[3], *cdvcm, *cdvm;
};

inline StateView make_view(void *base, const Layout &L)
{
    char *b = static_cast<char *>(base);
    auto f = [&](int k) { return reinterpret_cast<float *>(b + L.slot(k)); };
    auto u = [&](int k) { return reinterpret_cast<uint32_t *>(b + L.slot(k)); };
    StateView s;
    s.hdr = reinterpret_cast<SetHeader *>(b + L.hdr);
    s.mprefix = reinterpret_cast<double *>(b + L.mprefix);
    s.fctab = reinterpret_cast<double *>(b + L.fctab);
    s.lbtab = reinterpret_cast<float *>(b + L.lbtab);
    for (int a = 0; a < 3; ++a) {
        s.pos[a] = f(SL_POS + a);
        s.nrm[a] = f(SL_NRM + a);
        s.u[a] = f(SL_U + a);
        s.v[a] = f(SL_V + a);
        s.cb[a] = f(SL_CB + a);
    }
    s.r = f(SL_R);
    s.t = u(SL_T);
    s.nseen = u(SL_NSEEN);
    s.orig = u(SL_ORIG);
    s.cnt = u(SL_CNT);
    s.dec = u(SL_DEC);
    s.cand = u(SL_CAND);
    s.sq0 = f(SL_SQ);
    s.sq2 = reinterpret_cast<double2 *>(s.sq0);
    s.nch = L.nch;
    s.tau0 = f(SL_TAU);
    s.astride = (uint32_t)(L.stride / sizeof(float));
    s.F = reinterpret_cast<double *>(b + L.slot(SL_F));
    s.Fc = reinterpret_cast<double *>(b + L.slot(SL_FC));
    s.cdvcm = f(SL_CDVCM);
    s.cdvm = f(SL_CDVM);
    return s;
}

// Per-set record read by the batched gather (device table in the workspace).
struct SetDesc {
    char *state;             // state base
    uint64_t arr;            // byte offset of slot 0
    uint64_t stride;         // bytes per slot
    uint32_t H;
    uint32_t pay_off;        // first photon of the set in the combined payload
    uint32_t cell_base;      // first cell start of the set in the combined cell-start array
    uint32_t max_iters;
    uint64_t mprefix, fctab, lbtab, hdr;   // byte offsets in the state
    uint32_t q_off;          // first entry of the set in the batch's work list
    uint32_t max_cells;      // cell-count bound of the set's grid plan
};

// Blocks of one launch over several sets of a batch (a kernel argument): the i-th set of the launch
// owns blocks [pre[i], pre[i + 1]).
struct SetBlocks {
    int n;
    uint32_t pre[MAX_BATCH + 1];
};

// The launch's set of block b: the largest i with pre[i] <= b (binary search over the argument).
__device__ __forceinline__ int block_set(const SetBlocks &B, uint32_t b)
{
    int lo = 0, hi = B.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (B.pre[mid] <= b)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;     // keys per radix block
constexpr int SCAN_TILE = 4096;                    // counters per scan block
constexpr int SPLIT_TILE = 4096;                   // work-list entries per partition block
// sorted payload: one record of float4s per photon, (x, y, z, luminance), (R, G, B, dVCM) and, when a
// normal test or vertex merging reads it, (nx, ny, nz, dVM): 32 or 48 bytes
constexpr int PAY_VEC = 3;
__host__ __device__ constexpr int pay_rec(bool nrm_or_vcm) { return nrm_or_vcm ? 3 : 2; }
// photons of one gather launch: the byte offsets of its records fit 32 bits, and so does every cursor
// value a lane forms: a lane's cursor steps G records at a time and may pass the end of the last row
// by up to 63 records before it moves to the point at infinity, which follows the records
constexpr int64_t max_batch_photons(int rec) { return (int64_t)(0xFFFFFFFFull / (16ull * rec)) - 64; }

inline uint32_t max_cells_for(int64_t n_photons)
{
    int64_t mc = 4 * (n_photons > 1024 ? n_photons : 1024);
    if (mc > (int64_t)MAX_CELLS) mc = MAX_CELLS;
    return (uint32_t)mc;
}

// The grids of a batch's sets are built on up to GRID_STREAMS streams at once (the sets are
// independent until the gather); each stream has its own sort scratch. Three: with the critical
// values' stream that makes four streams, as many as HIP gives a process hardware queues by default;
// a fourth grid stream shares a queue with another, whose work then runs behind its own.
constexpr int GRID_STREAMS = 3;

struct SortScratch {
    size_t keyA = 0, keyB = 0, valA = 0, valB = 0, hist = 0, part = 0, part3 = 0;
};

// Workspace of one batched iteration (or of the kernel ordering in hk_set_kernels).
struct WsLayout {
    int n_sets = 0;
    int ngs = 1;              // grid streams of the batch: min(sets, GRID_STREAMS)
    int64_t n_total = 0, h_total = 0, n_max = 0;
    int64_t pstride = 0;      // payload records: the batch's photons, then one point at infinity
    SortScratch sort[GRID_STREAMS];
    size_t cstart = 0, pay = 0;
    size_t flag = 0, ids = 0, tiles = 0, heavy = 0, light = 0, lcost = 0, counts = 0, desc = 0;
    uint32_t pay_off[MAX_BATCH] = {}, cell_base[MAX_BATCH] = {}, max_cells[MAX_BATCH] = {};
    uint32_t q_off[MAX_BATCH] = {};
    size_t total = 0;
};

inline WsLayout make_ws_layout(int n_sets, const int64_t *n_photons, const int64_t *n_kernels)
{
    WsLayout W;
    W.n_sets = n_sets;
    int64_t nmax = 1, cells = 0;
    // with more than MAX_BATCH sets only the sizes are meaningful (a bound for any batch of them)
    for (int s = 0; s < n_sets; ++s) {
        const uint32_t mc = max_cells_for(n_photons[s]);
        if (s < MAX_BATCH) {
            W.pay_off[s] = (uint32_t)W.n_total;
            W.q_off[s] = (uint32_t)W.h_total;
            W.cell_base[s] = (uint32_t)cells;
            W.max_cells[s] = mc;
        }
        cells += (int64_t)mc + 2;
        W.n_total += n_photons[s];
        W.h_total += n_kernels[s];
        if (n_photons[s] > nmax) nmax = n_photons[s];
        if (n_kernels[s] > nmax) nmax = n_kernels[s];
    }
    W.n_max = nmax;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    W.ngs = n_sets < GRID_STREAMS ? (n_sets > 0 ? n_sets : 1) : GRID_STREAMS;
    for (int g = 0; g < W.ngs; ++g) {
        SortScratch &S = W.sort[g];
        S.keyA = take(4 * (size_t)nmax);
        S.keyB = take(4 * (size_t)nmax);
        S.valA = take(4 * (size_t)nmax);
        S.valB = take(4 * (size_t)nmax);
        const int64_t nblk = cdiv(nmax, RS_TILE);
        S.hist = take(4 * (size_t)(256 * (RS_TILE / 64) * nblk));      // per digit and wavefront chunk
        S.part = take(4 * (size_t)(cdiv(256 * (RS_TILE / 64) * nblk, SCAN_TILE) + 1));   // its scan's partials
        S.part3 = take(4 * (size_t)(cdiv((int64_t)MAX_CELLS + 2, SCAN_TILE) + 1));
    }
    W.cstart = take(4 * (size_t)(cells + 1));
    W.pstride = W.n_total + 1;
    W.pay = take(16 * (size_t)W.pstride * PAY_VEC + 256);      // records of up to PAY_VEC float4s
    const size_t hk = 4 * (size_t)(W.h_total + 1);
    W.flag = take(hk);
    W.ids = take(hk);
    W.tiles = take(4 * (size_t)(cdiv(W.h_total + 1, SPLIT_TILE) + 3));   // two gather phases' tiles
    W.heavy = take(hk);
    W.light = take(hk);
    W.lcost = take(hk);
    W.counts = take(64);
    W.desc = take(sizeof(SetDesc) * MAX_BATCH);
    W.total = off;
    return W;
}

// ---------------------------------------------------------------------------------------------
// Device arithmetic shared by the kernels (float32, explicit operation order, no contraction)
// ---------------------------------------------------------------------------------------------

// Tangent frame of a unit normal: Duff et al., "Building an Orthonormal Basis, Revisited" (2017).
__device__ __forceinline__ void onb(float x, float y, float z, float *u, float *v)
{
    float sgn = copysignf(1.0f, z);
    float a = -1.0f / (sgn + z);
    float b = (x * y) * a;
    u[0] = 1.0f + ((sgn * x) * x) * a;
    u[1] = sgn * b;
    u[2] = -(sgn * x);
    v[0] = b;
    v[1] = sgn + (y * y) * a;
    v[2] = -y;
}

// Group index of y = (yu, yv) at squared distance d2 < r2: annulus (2 d2 >= r2) x sector, sector s
// covering polar angles [60 s, 60 (s+1)) degrees from +u, centre in sector 0 (Sec. 3.2.1).
__device__ __forceinline__ int group_of(float yu, float yv, float d2, float r2)
{
    const float s3 = 1.7320508075688772f;
    const int ann = (d2 + d2 >= r2) ? 6 : 0;
    const float a = fmaf(-s3, yu, yv);
    const float b = fmaf(s3, yu, yv);
    const bool upper = (yv > 0.0f) | ((yv == 0.0f) & (yu >= 0.0f));
    const int su = (a < 0.0f) ? 0 : ((b > 0.0f) ? 1 : 2);
    const int sl = (a > 0.0f) ? 3 : ((b < 0.0f) ? 4 : 5);
    int s = upper ? su : sl;
    s = ((yu == 0.0f) & (yv == 0.0f)) ? 0 : s;
    return ann + s;
}

__device__ __forceinline__ float luminance(float R, float G, float B)
{
    return fmaf(0.0722f, B, fmaf(0.7152f, G, 0.2126f * R));
}

// Compensated float32 accumulation into a pair (s, c) that stands for s + c: Knuth's TwoSum gives
// the rounding error e of s + x exactly (s + x = t + e), and c collects those errors (the Neumaier
// form of compensated summation). Unlike the classic Kahan update, the error of forming x - c is not
// lost, so the pair tracks the exact sum to about n u^2 of its magnitude instead of u per term.
__device__ __forceinline__ void acc2(float &s, float &c, float x)
{
    const float t = s + x;
    const float z = t - s;
    const float e = (s - (t - z)) + (x - z);
    s = t;
    c += e;
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

// Cells [x0, x1] of the stencil row (cy, cz) that can hold a light vertex within r of p, a subrange of
// the stencil's [c0x, c1x]: every point of the row's y and z slabs lies at least dy and dz from p,
// so such a vertex has |x - p_x| < sqrt(r^2 - dy^2 - dz^2). The slab distances are reduced by the
// rounding margin mg and the half-width grown by it, so no vertex within r is ever left out; the
// rows keep their order, so the in-disk photons reach the sums in the same order as with the full
// stencil. wy, wz are the cell widths 1 / cell_inv. False when no vertex of the row can lie within r.
__device__ __forceinline__ bool row_span(const SetHeader *hdr, const float p[3], float r, float mg, float wy,
                                         float wz, int cy, int cz, int c0x, int c1x, int &x0, int &x1)
{
    float h2 = r * r;
    const int c[3] = {0, cy, cz};
    const float w[3] = {0.0f, wy, wz};
#pragma unroll
    for (int a = 1; a < 3; ++a) {
        const float lo = fmaf((float)c[a], w[a], hdr->dom_lo[a]);
        const float d = fmaxf(fmaxf(lo - p[a], p[a] - (lo + w[a])) - mg, 0.0f);
        h2 = fmaf(-d, d, h2);
    }
    if (!(h2 >= 0.0f)) return false;
    const float h = sqrtf(h2) + mg;
    const float f0 = floorf((p[0] - h - hdr->dom_lo[0]) * hdr->cell_inv[0]);
    const float f1 = floorf((p[0] + h - hdr->dom_lo[0]) * hdr->cell_inv[0]);
    x0 = (int)fminf(fmaxf(f0, (float)c0x), (float)c1x);
    x1 = (int)fminf(fmaxf(f1, (float)c0x), (float)c1x);
    return f1 >= (float)c0x && f0 <= (float)c1x;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

// Exclusive scan over a 256-thread block; *total receives the block sum.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t wsum[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i < w) off += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

// Radius histogram bin: floor(-4 log2(r / r1)) clamped to the table.
__device__ __forceinline__ int radius_bin(float r, float r1)
{
    const float b = floorf(-4.0f * log2f(r / r1));
    return (b >= 0.0f) ? ((b < (float)(RHIST_BINS - 1)) ? (int)b : RHIST_BINS - 1) : 0;
}


}  // namespace hk

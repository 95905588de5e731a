// Internal definitions of libhk: per-set state layout, device helpers, kernel launch declarations.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "hk.h"

namespace hk {

constexpr int NG = 12;              // 2 annuli x 6 sectors (Sec. 6.1.1)
constexpr int NSQ = 4 * NG;         // per group: S, comp(S), Q, comp(Q)
constexpr int RHIST_BINS = 64;      // radius histogram: bin = floor(-4 log2(r / r1))
constexpr uint32_t KEY_OUTSIDE = 0xFFFFFFu;   // cell key of a photon outside the grid domain
constexpr uint32_t MAX_CELLS = 0xFFFFF0u;     // keys fit 24 bits: three 8-bit radix passes
constexpr int WAVE = 64;            // wavefront width of gfx950
constexpr int G_LIGHT = 16;         // lanes per kernel in a light work item (4 kernels per wave)
constexpr int G_HEAVY = 64;         // lanes per kernel in a heavy work item (1 kernel per wave)
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
    int32_t pad[4];
    // running totals since hk_set_kernels (gather launches, in-disk pairs, lane x photon tests)
    unsigned long long n_launch;
    unsigned long long n_pairs;
    unsigned long long n_cand;
};

// Offsets (bytes) of every array of a set's state; each array is 256-byte aligned.
struct Layout {
    int64_t H = 0;
    int max_iters = 0;
    size_t hdr = 0, mprefix = 0, fctab = 0;
    size_t pos[3] = {}, nrm[3] = {}, u[3] = {}, v[3] = {};
    size_t r = 0, t = 0, nseen = 0, orig = 0, cnt = 0, dec = 0;
    size_t sq[NSQ * 3] = {};    // luminance test uses the first NSQ; per-channel test all 3 x NSQ
    size_t tau[6] = {};         // R, comp R, G, comp G, B, comp B
    size_t F = 0, Fc = 0;
    size_t cb[3] = {}, cdvcm = 0, cdvm = 0;
    size_t total = 0;
};

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline Layout make_layout(int64_t H, int max_iters, bool rgb_stats)
{
    Layout L;
    L.H = H;
    L.max_iters = max_iters;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    L.hdr = take(sizeof(SetHeader));
    L.mprefix = take(sizeof(double) * (max_iters + 2));
    L.fctab = take(sizeof(double) * (max_iters + 2));
    const size_t f = sizeof(float) * (size_t)H;
    for (int a = 0; a < 3; ++a) L.pos[a] = take(f);
    for (int a = 0; a < 3; ++a) L.nrm[a] = take(f);
    for (int a = 0; a < 3; ++a) L.u[a] = take(f);
    for (int a = 0; a < 3; ++a) L.v[a] = take(f);
    L.r = take(f);
    L.t = take(f);
    L.nseen = take(f);
    L.orig = take(f);
    L.cnt = take(f);
    L.dec = take(f);
    const int nsq = rgb_stats ? 3 * NSQ : NSQ;
    for (int i = 0; i < nsq; ++i) L.sq[i] = take(f);
    for (int i = 0; i < 6; ++i) L.tau[i] = take(f);
    L.F = take(2 * f);
    L.Fc = take(2 * f);
    for (int a = 0; a < 3; ++a) L.cb[a] = take(f);
    L.cdvcm = take(f);
    L.cdvm = take(f);
    L.total = off;
    return L;
}

// Device view of one set's state (raw pointers into the caller's buffer).
struct StateView {
    SetHeader *hdr;
    double *mprefix;     // mprefix[i] = sum of J over iterations 1..i
    double *fctab;       // fctab[t] = critical value for t kept iterations
    float *pos[3], *nrm[3], *u[3], *v[3];
    float *r;
    uint32_t *t, *nseen, *orig, *cnt, *dec;
    float *sq[NSQ * 3];
    float *tau[6];
    double *F, *Fc;
    float *cb[3], *cdvcm, *cdvm;
};

inline StateView make_view(void *base, const Layout &L)
{
    char *b = static_cast<char *>(base);
    StateView s;
    s.hdr = reinterpret_cast<SetHeader *>(b + L.hdr);
    s.mprefix = reinterpret_cast<double *>(b + L.mprefix);
    s.fctab = reinterpret_cast<double *>(b + L.fctab);
    for (int a = 0; a < 3; ++a) {
        s.pos[a] = reinterpret_cast<float *>(b + L.pos[a]);
        s.nrm[a] = reinterpret_cast<float *>(b + L.nrm[a]);
        s.u[a] = reinterpret_cast<float *>(b + L.u[a]);
        s.v[a] = reinterpret_cast<float *>(b + L.v[a]);
        s.cb[a] = reinterpret_cast<float *>(b + L.cb[a]);
    }
    s.r = reinterpret_cast<float *>(b + L.r);
    s.t = reinterpret_cast<uint32_t *>(b + L.t);
    s.nseen = reinterpret_cast<uint32_t *>(b + L.nseen);
    s.orig = reinterpret_cast<uint32_t *>(b + L.orig);
    s.cnt = reinterpret_cast<uint32_t *>(b + L.cnt);
    s.dec = reinterpret_cast<uint32_t *>(b + L.dec);
    for (int i = 0; i < NSQ * 3; ++i) s.sq[i] = L.sq[i] ? reinterpret_cast<float *>(b + L.sq[i]) : nullptr;
    for (int i = 0; i < 6; ++i) s.tau[i] = reinterpret_cast<float *>(b + L.tau[i]);
    s.F = reinterpret_cast<double *>(b + L.F);
    s.Fc = reinterpret_cast<double *>(b + L.Fc);
    s.cdvcm = reinterpret_cast<float *>(b + L.cdvcm);
    s.cdvm = reinterpret_cast<float *>(b + L.cdvm);
    return s;
}

// Workspace carve-up for one set's iteration (or for the kernel ordering in hk_set_kernels).
struct WsLayout {
    int64_t max_photons = 0, max_kernels = 0;
    uint32_t max_cells = 0;
    size_t keyA = 0, keyB = 0, valA = 0, valB = 0, hist = 0, part = 0, cstart = 0, pay = 0;
    size_t flag = 0, offs = 0, part2 = 0, part3 = 0, heavy = 0, light = 0, counts = 0;
    size_t total = 0;
};

constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;     // keys per radix block
constexpr int SCAN_TILE = 4096;                    // counters per scan block
// sorted payload, three float4 per photon: (x, y, z, luminance), (nx, ny, nz, dVM), (R, G, B, dVCM)
constexpr int PAY_VEC = 3;

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline WsLayout make_ws_layout(int64_t max_photons, int64_t max_kernels)
{
    WsLayout W;
    int64_t n = max_photons > max_kernels ? max_photons : max_kernels;
    if (n < 1) n = 1;
    W.max_photons = max_photons;
    W.max_kernels = max_kernels;
    int64_t mc = 4 * (max_photons > 1024 ? max_photons : 1024);
    if (mc > (int64_t)MAX_CELLS) mc = MAX_CELLS;
    W.max_cells = (uint32_t)mc;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    W.keyA = take(4 * (size_t)n);
    W.keyB = take(4 * (size_t)n);
    W.valA = take(4 * (size_t)n);
    W.valB = take(4 * (size_t)n);
    int64_t nblk = cdiv(n, RS_TILE);
    W.hist = take(4 * (size_t)(256 * nblk));
    W.part = take(4 * (size_t)(cdiv(256 * nblk, SCAN_TILE) + 1));
    W.cstart = take(4 * (size_t)(W.max_cells + 2));
    W.part3 = take(4 * (size_t)(cdiv((int64_t)W.max_cells + 1, SCAN_TILE) + 1));
    W.pay = take(16 * (size_t)max_photons * PAY_VEC + 256);
    const size_t hk = 4 * (size_t)(max_kernels + 1);
    W.flag = take(hk);
    W.offs = take(hk);
    W.part2 = take(4 * (size_t)(cdiv(max_kernels + 1, SCAN_TILE) + 1));
    W.heavy = take(hk);
    W.light = take(hk);
    W.counts = take(64);
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

// Compensated (Kahan) accumulation: (s - c) tracks the exact running sum to O(n u^2).
__device__ __forceinline__ void kahan(float &s, float &c, float x)
{
    const float y = x - c;
    const float t = s + y;
    c = (t - s) - y;
    s = t;
}

// Radius histogram bin: floor(-4 log2(r / r1)) clamped to the table.
__device__ __forceinline__ int radius_bin(float r, float r1)
{
    const float b = floorf(-4.0f * log2f(r / r1));
    return (b >= 0.0f) ? ((b < (float)(RHIST_BINS - 1)) ? (int)b : RHIST_BINS - 1) : 0;
}


}  // namespace hk

// Launch descriptors shared by the host API and the kernel files.
#pragma once
#include "hk_internal.h"

namespace hk {

struct PhotonSrc {
    const float *pos[3];
    const float *nrm[3];
    const float *flux[3];
    const float *mis[3];
};

struct KernelSrc {
    const float *pos[3];
    const float *nrm[3];
    const float *r_init;
    const float *cam_beta[3];
    const float *cam_mis[3];
};

// Grid build of one set; its payload records go to records pay_off.. of the batch's payload, its cell
// starts (set-local photon positions) to cstart.
struct GridLaunch {
    SetHeader *hdr;
    PhotonSrc src;
    int64_t n;
    uint32_t *keyA, *keyB, *valA, *valB, *hist, *part, *part3, *cstart;
    float4 *pay;             // the batch's payload: record q at pay + q * rec
    int rec;                 // float4s per record (pay_rec of the batch)
    int64_t pay_off;         // the set's first photon in the batch's payload
    uint32_t ncells_bound;   // cells of the plan never exceed this (workspace capacity)
};

struct InitLaunch {
    StateView st;
    KernelSrc src;
    int64_t n;
    int max_iters;
    float r1;
    float r_floor;           // smallest admissible caller radius: the first lower bound, r_min
    int vcm;
    uint32_t *keyA, *keyB, *valA, *valB, *hist, *part;
};

// Work-list construction, per set: cost of each kernel into flag/offs/ids at q_off.
struct ListLaunch {
    int64_t H;
    SetHeader *hdr;
    const uint32_t *cstart;
    const float *kp[3];
    const float *r;
    const uint32_t *cand, *dec;  // the last iteration's candidate tests and shrink decisions
    float k2;                    // shrink factor squared (area ratio of a shrink)
    uint32_t heavy_cost;
    uint32_t set_slot;       // index of the set in the batch
    uint32_t q_base;         // the set's first entry in the batch's work list
    uint32_t *flag, *ids;        // flag: each kernel's expected cost
    uint32_t *tile_heavy;    // heavy kernels per SPLIT_TILE entries of the work list (zeroed before)
};

// Everything the batched gather / test / update kernel needs besides the per-set table.
struct BatchArgs {
    const SetDesc *desc;     // per-set table (device)
    const float4 *pay;       // combined payload records (pay_rec(NRM || VCM) float4s each)
    uint32_t pstride;        // records: the batch's photons, then one point at infinity
    const uint32_t *cstart;  // combined cell starts (set-local positions)
    const uint32_t *heavy, *light, *counts;   // work list, entries (set << Q_BITS) | kernel
    float k;
    float cos_min;
    int lanes_light, lanes_heavy;
};

// Learned radius proposal: 36 -> 64 -> 64 -> 1 perceptron. Parameter vector: W1 (36 x 64, row =
// input), b1, W2 (64 x 64, row = input), b2, w3, b3.
constexpr int MLP_IN = 36, MLP_INP = 64, MLP_H = 64;
constexpr int MLP_OFF_W1 = 0, MLP_OFF_B1 = MLP_IN * MLP_H, MLP_OFF_W2 = MLP_OFF_B1 + MLP_H;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_H * MLP_H, MLP_OFF_W3 = MLP_OFF_B2 + MLP_H, MLP_OFF_B3 = MLP_OFF_W3 + MLP_H;
constexpr int MLP_P = MLP_OFF_B3 + 1;              // 6593 parameters
constexpr int MLP_PP = 6656;                       // parameters + squared error, rounded up
constexpr int MLP_MAX_WG = 1024;                   // workgroups of a gradient launch

// Device view of a network's state: float32 master parameters, Adam moments (float64), bfloat16
// copies of the weights as the matrix cores read them (W1 padded to 64 input rows), step count.
struct MlpView {
    float *theta;
    double *m, *v;
    uint16_t *w1b, *w2b, *w3b;
    int64_t *step;
};

struct MlpLayout {
    size_t theta = 0, m = 0, v = 0, w1b = 0, w2b = 0, w3b = 0, step = 0, total = 0;
};

inline MlpLayout mlp_layout()
{
    MlpLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    L.theta = take(sizeof(float) * MLP_PP);
    L.m = take(sizeof(double) * MLP_PP);
    L.v = take(sizeof(double) * MLP_PP);
    L.w1b = take(2 * MLP_INP * MLP_H);
    L.w2b = take(2 * MLP_H * MLP_H);
    L.w3b = take(2 * MLP_H);
    L.step = take(sizeof(int64_t));
    L.total = off;
    return L;
}

inline MlpView mlp_view(void *base)
{
    char *b = static_cast<char *>(base);
    const MlpLayout L = mlp_layout();
    MlpView M;
    M.theta = reinterpret_cast<float *>(b + L.theta);
    M.m = reinterpret_cast<double *>(b + L.m);
    M.v = reinterpret_cast<double *>(b + L.v);
    M.w1b = reinterpret_cast<uint16_t *>(b + L.w1b);
    M.w2b = reinterpret_cast<uint16_t *>(b + L.w2b);
    M.w3b = reinterpret_cast<uint16_t *>(b + L.w3b);
    M.step = reinterpret_cast<int64_t *>(b + L.step);
    return M;
}

int mlp_grid(int64_t n);
void launch_mlp_set(const MlpView &M, const float *theta, hipStream_t s);
void launch_mlp_forward(const MlpView &M, const uint16_t *feat, int64_t n, float *y, hipStream_t s);
void launch_mlp_grad(const MlpView &M, const uint16_t *feat, const float *label, int64_t n, float *part, float *grad,
                     hipStream_t s);
void launch_mlp_adam(const MlpView &M, const float *grad, float lr, hipStream_t s);
void launch_features(const StateView &st, int64_t H, const uint32_t *cstart, const float4 *pay, int rec,
                     bool nrm_test, float cos_min, float it_code, uint16_t *feat, uint32_t *counts, hipStream_t s);
void launch_propose(const StateView &st, int64_t H, const float *y, float margin, hipStream_t s);

// first_hist_done: the first pass's histogram is already in `hist` (written with the keys).
void radix_sort(uint32_t *kA, uint32_t *vA, uint32_t *kB, uint32_t *vB, int64_t n, int bits, uint32_t *hist,
                uint32_t *part, hipStream_t s, uint32_t **kres, uint32_t **vres, bool inverse, bool first_hist_done);
void build_grid(const GridLaunch &g, hipStream_t s);
void init_set(const InitLaunch &g, hipStream_t s);
void excl_scan(uint32_t *d, int64_t len, uint32_t *part, hipStream_t s, const uint32_t *dlen = nullptr,
               int extra = 0);
// Per iteration, one block per set of a batch (the set table must be on the device): advance the
// iteration, append J, plan the grid.
void launch_plan_batch(const SetDesc *desc, int nb, const double *J, float cell_scale, float quantile,
                       hipStream_t s);
void launch_plan_fixed(SetHeader *hdr, float cell, uint32_t max_cells, hipStream_t s);
// Critical values of a batch's sets in one launch (the set table on the device); all[k]: recompute
// every kept-iteration count of set k, else only the new one.
void launch_fcrit(const SetDesc *desc, int nb, const uint8_t *all, int max_iters, double alpha_f, hipStream_t s);
// Expected cost of every kernel of sets k0 .. k1-1 of a batch (one gather phase, whose work list
// starts at entry q0): flags, entries and the heavy counts per tile.
struct CostBatch {
    const SetDesc *desc;
    int k0, k1;
    uint32_t q0;
    const uint32_t *cstart;      // the batch's cell starts
    uint32_t *flag, *ids;        // the batch's work-list arrays
    uint32_t *tile_heavy;        // the phase's heavy counts per tile (zeroed before)
    float k2;
    uint32_t heavy_cost;
};
void launch_cost_batch(const CostBatch &c, const uint32_t *H, hipStream_t s);   // H: hit points per batch slot
void launch_split(uint32_t *cost, uint32_t *ids, int64_t n, uint32_t heavy_cost, const uint32_t *tile_heavy,
                  uint32_t *heavy, uint32_t *light, uint32_t *lcost, uint32_t *counts, float4 *sentinel,
                  hipStream_t s);
void launch_zero(uint32_t *p, int64_t n, hipStream_t s);
void launch_upload(void *dst, const void *src, size_t bytes, hipStream_t s);   // bytes: multiple of 4
void launch_gather(const BatchArgs &a, int64_t h_total, bool nrm, bool vcm, int nch, hipStream_t s);
void launch_tally(const SetDesc *desc, const uint32_t *H, int nb, hipStream_t s);   // H: hit points per set

// light-vertex generation for the box scene (one thread per slot)
struct EmitLaunch {
    const SetHeader *hdr;    // the set's header: its iteration count picks the random stream
    float L[3], C[3], R, power;
    uint32_t key0, key1, set_id;
    int64_t J;
    float *pos[3], *nrm[3], *flux[3];
    float *mis[3];           // vertex-merging partials (dVCM, dVC, dVM), or all NULL
};
void launch_emit_box(const EmitLaunch &e, hipStream_t s);

// vertex connection of every camera vertex to the box scene's point light (next-event estimation),
// weighted against merging and added to the set's running estimate
struct ConnectLaunch {
    StateView st;
    int64_t H;
    float L[3], C[3], R, intensity, Jf;
};
void launch_connect_box(const ConnectLaunch &c, hipStream_t s);

}  // namespace hk

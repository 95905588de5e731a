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

// Grid build of one set; its payload goes to pay + pay_off in each of the PAY_VEC planes of
// pstride photons, its cell starts (set-local photon positions) to cstart.
struct GridLaunch {
    SetHeader *hdr;
    PhotonSrc src;
    int64_t n;
    uint32_t *keyA, *keyB, *valA, *valB, *hist, *part, *part3, *cstart;
    float4 *pay;
    int64_t pstride;
    uint32_t ncells_bound;   // cells of the plan never exceed this (workspace capacity)
};

struct InitLaunch {
    StateView st;
    KernelSrc src;
    int64_t n;
    int max_iters;
    float r1;
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
    uint32_t heavy_cost;
    uint32_t set_slot;       // index of the set in the batch
    uint32_t *flag, *offs, *ids;
};

// Everything the batched gather / test / update kernel needs besides the per-set table.
struct BatchArgs {
    const SetDesc *desc;     // per-set table (device)
    const float4 *pay;       // combined payload: plane v at pay + v * pstride
    uint32_t pstride;
    const uint32_t *cstart;  // combined cell starts (set-local positions)
    const uint32_t *heavy, *light, *counts;   // work list, entries (set << Q_BITS) | kernel
    float k;
    float cos_min;
    int lanes_light, lanes_heavy;
};

void radix_sort(uint32_t *kA, uint32_t *vA, uint32_t *kB, uint32_t *vB, int64_t n, int bits, uint32_t *hist,
                uint32_t *part, hipStream_t s, uint32_t **kres, uint32_t **vres);
void build_grid(const GridLaunch &g, hipStream_t s);
void init_set(const InitLaunch &g, hipStream_t s);
void excl_scan(uint32_t *d, int64_t len, uint32_t *part, hipStream_t s);
void launch_plan(SetHeader *hdr, double *mprefix, double J, float cell_scale, float quantile, uint32_t max_cells,
                 hipStream_t s);
void launch_fcrit(const SetHeader *hdr, double *fctab, const double *mprefix, int max_iters, bool all, double alpha_f,
                  hipStream_t s);
void launch_cost(const ListLaunch &l, hipStream_t s);
void launch_split(uint32_t *flag, uint32_t *offs, uint32_t *ids, int64_t n, uint32_t *part, uint32_t *heavy,
                  uint32_t *light, uint32_t *counts, hipStream_t s);
void launch_upload(void *dst, const void *src, size_t bytes, hipStream_t s);   // bytes: multiple of 4
void launch_gather(const BatchArgs &a, int64_t h_total, bool nrm, bool vcm, hipStream_t s);
void launch_tally(const SetDesc *desc, const uint32_t *ids, int64_t h_total, hipStream_t s);

}  // namespace hk

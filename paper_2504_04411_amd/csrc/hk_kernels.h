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

struct GridLaunch {
    SetHeader *hdr;
    PhotonSrc src;
    int64_t n;
    uint32_t *keyA, *keyB, *valA, *valB, *hist, *part, *part3, *cstart;
    float4 *pay;             // payload, PAY_VEC float4 rows of pstride photons
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
    int nsq;
    uint32_t *keyA, *keyB, *valA, *valB, *hist, *part;
};

// Everything the fused gather / test / update kernel reads or writes for one set.
struct GatherArgs {
    int64_t H;
    SetHeader *hdr;
    const uint32_t *cstart;
    const float4 *payA, *payB, *payC;
    uint32_t npay;           // photons in each payload plane (< 2^28: 32-bit byte offsets)
    const float *kp[3], *kn[3], *ku[3], *kv[3];
    float *r;
    uint32_t *t, *nseen, *cnt, *dec;
    float *sq0;              // group sums: array i at sq0 + i * astride (i = 4 g + {S, comp S, Q, comp Q})
    float *tau0;             // estimate: array c at tau0 + c * astride (R, comp R, G, comp G, B, comp B)
    uint32_t astride;        // floats between consecutive per-kernel arrays of the state
    double *F, *Fc;
    const float *cb[3], *cdvcm, *cdvm;
    const double *fctab, *mprefix;
    int iter;
    float Jf;
    float lb;
    float k;
    float cos_min;
    float r1;
    // work list: heavy kernels first, then light kernels; lanes per kernel for each kind
    const uint32_t *heavy, *light, *counts;
    int lanes_light, lanes_heavy;
};

// Work-list construction for one set's gather.
struct ListLaunch {
    int64_t H;
    const SetHeader *hdr;
    const uint32_t *cstart;
    const float *kp[3];
    const float *r;
    uint32_t heavy_cost;
    uint32_t *flag, *offs, *part2, *heavy, *light, *counts;
};

void radix_sort(uint32_t *kA, uint32_t *vA, uint32_t *kB, uint32_t *vB, int64_t n, int bits, uint32_t *hist,
                uint32_t *part, hipStream_t s, uint32_t **kres, uint32_t **vres);
void build_grid(const GridLaunch &g, hipStream_t s);
void init_set(const InitLaunch &g, hipStream_t s);
void launch_plan(SetHeader *hdr, double *mprefix, int iter, double J, float cell_scale, float quantile,
                 uint32_t max_cells, hipStream_t s);
void launch_fcrit(double *fctab, const double *mprefix, int iter, int t_lo, int t_hi, double alpha_f,
                  hipStream_t s);
void build_work_list(const ListLaunch &l, hipStream_t s);
void launch_gather(const GatherArgs &a, bool nrm, bool vcm, hipStream_t s);
void excl_scan(uint32_t *d, int64_t len, uint32_t *part, hipStream_t s);

}  // namespace hk

// Learned radius proposal (an addition to the paper's method): ring-count features of the hit points,
// a 36 -> 64 -> 64 -> 1 ReLU perceptron on bfloat16 matrix cores (forward, back-propagation, Adam),
// and the proposal r = clamp(r1 exp(y), lb, r_current) written into a set's state. The F-test of
// the estimator stays in charge afterwards: it can only shrink the proposed radii further.
//
// Matrix products use v_mfma_f32_16x16x32_bf16 (gfx950): a wavefront multiplies a 16 x 32 bfloat16
// tile by a 32 x 16 tile into 16 x 16 float32. Lane l supplies row (l mod 16) of A and column
// (l mod 16) of B, each with the 8 consecutive k = 8 (l / 16) .. + 7, and receives rows
// 4 (l / 16) .. + 3 of output column (l mod 16). Operands are staged in LDS; a transposed operand
// is the same tile read with swapped strides, so the backward products need no extra copies.
//
// A workgroup (4 wavefronts) takes blocks of 64 samples; each wavefront owns one 16-row band of
// every 64 x 64 product. Rounding points (bfloat16 after each ReLU and for the back-propagated
// errors entering a product; float32 accumulation) are the ones the CPU reference emulates.
#include <math.h>

#include "hk_internal.h"
#include "hk_kernels.h"

namespace hk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int LD = 72;              // LDS row stride (bfloat16 elements) of a 64 x 64 tile
constexpr int SB = 64;              // samples per block

__device__ __forceinline__ uint16_t f2bf(float x)
{
    uint32_t b = __float_as_uint(x);
    b += 0x7FFFu + ((b >> 16) & 1u);        // round to nearest even
    return (uint16_t)(b >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// acc += A(m0 + 0..15, 0..K) B(0..K, n0 + 0..15) with A(m, k) = a[m sam + k sak], B(k, n) = b[k sbk + n sbn].
__device__ __forceinline__ f32x4 mma_tile(const uint16_t *a, int sam, int sak, const uint16_t *b, int sbk, int sbn,
                                          int m0, int n0, int K, f32x4 acc)
{
    const int lane = threadIdx.x & 63, r = lane & 15, g = lane >> 4;
    for (int k0 = 0; k0 < K; k0 += 32) {
        u16x8 va, vb;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int k = k0 + 8 * g + e;
            va[e] = a[(m0 + r) * sam + k * sak];
            vb[e] = b[k * sbk + (n0 + r) * sbn];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, va), __builtin_bit_cast(bf16x8, vb),
                                                      acc, 0, 0, 0);
    }
    return acc;
}

struct MlpLds {
    uint16_t W1[MLP_INP * LD];       // [input][hidden]
    uint16_t W2[MLP_H * LD];         // [input][hidden]
    uint16_t X[SB * LD];             // [sample][input]
    uint16_t H1[SB * LD];            // [sample][hidden]; later the back-propagated error of layer 1
    uint16_t H2[SB * LD];            // [sample][hidden]; later the back-propagated error of layer 2
    float b1[MLP_H], b2[MLP_H], w3[MLP_H];
    float y[SB], dy[SB];
    float red[4];
};

__device__ void load_weights(const MlpView &M, MlpLds &L)
{
    for (int i = threadIdx.x; i < MLP_INP * MLP_H; i += 256) {
        const int r = i / MLP_H, c = i % MLP_H;
        L.W1[r * LD + c] = M.w1b[i];
        L.W2[r * LD + c] = M.w2b[i];
    }
    if (threadIdx.x < MLP_H) {
        const int h = threadIdx.x;
        L.b1[h] = M.theta[MLP_OFF_B1 + h];
        L.b2[h] = M.theta[MLP_OFF_B2 + h];
        L.w3[h] = bf2f(M.w3b[h]);
    }
}

// Forward pass of one block (samples s0 .. s0 + ns - 1); leaves H1, H2 in LDS and y (float32).
__device__ void forward_block(const MlpView &M, MlpLds &L, const uint16_t *feat, int64_t s0, int ns)
{
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
    for (int i = tid; i < SB * MLP_INP; i += 256) {
        const int s = i / MLP_INP, c = i % MLP_INP;
        uint16_t v = 0;
        if (s < ns && c < MLP_IN) v = feat[(s0 + s) * MLP_IN + c];
        L.X[s * LD + c] = v;
    }
    __syncthreads();
    // layer 1: Z1 = X W1 + b1; this wavefront's samples 16 w .. 16 w + 15
    for (int nt = 0; nt < 4; ++nt) {
        f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
        z = mma_tile(L.X, LD, 1, L.W1, LD, 1, 16 * w, 16 * nt, MLP_INP, z);
        const int h = 16 * nt + r;
#pragma unroll
        for (int e = 0; e < 4; ++e) L.H1[(16 * w + 4 * g + e) * LD + h] = f2bf(fmaxf(z[e] + L.b1[h], 0.0f));
    }
    __syncthreads();
    for (int nt = 0; nt < 4; ++nt) {
        f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
        z = mma_tile(L.H1, LD, 1, L.W2, LD, 1, 16 * w, 16 * nt, MLP_H, z);
        const int h = 16 * nt + r;
#pragma unroll
        for (int e = 0; e < 4; ++e) L.H2[(16 * w + 4 * g + e) * LD + h] = f2bf(fmaxf(z[e] + L.b2[h], 0.0f));
    }
    __syncthreads();
    // output: 4 threads per sample, 16 hidden units each, then a 4-lane sum
    {
        const int s = tid >> 2, q = tid & 3;
        float acc = 0.0f;
#pragma unroll
        for (int h = 16 * q; h < 16 * q + 16; ++h) acc += bf2f(L.H2[s * LD + h]) * L.w3[h];
        acc += __shfl_xor(acc, 1, WAVE);
        acc += __shfl_xor(acc, 2, WAVE);
        if (q == 0) L.y[s] = acc + M.theta[MLP_OFF_B3];
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void mlp_forward_kernel(MlpView M, const uint16_t *feat, int64_t n, float *y)
{
    __shared__ MlpLds L;
    load_weights(M, L);
    __syncthreads();
    for (int64_t s0 = (int64_t)blockIdx.x * SB; s0 < n; s0 += (int64_t)gridDim.x * SB) {
        const int ns = (int)min((int64_t)SB, n - s0);
        forward_block(M, L, feat, s0, ns);
        if ((int)threadIdx.x < ns) y[s0 + threadIdx.x] = L.y[threadIdx.x];
        __syncthreads();
    }
}

// Gradient of the mean squared error over n samples: every workgroup writes the sum over its
// blocks to its row of `part` (MLP_PP floats: the parameters' gradients, then the squared error).
__global__ __launch_bounds__(256) void mlp_grad_kernel(MlpView M, const uint16_t *feat, const float *label, int64_t n,
                                                       float inv_n, float *part)
{
    __shared__ MlpLds L;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
    load_weights(M, L);
    __syncthreads();
    f32x4 gW1[4], gW2[4];
    for (int t = 0; t < 4; ++t) {
        gW1[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        gW2[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    }
    float gb1 = 0.0f, gb2 = 0.0f, gw3 = 0.0f, gb3 = 0.0f, sq = 0.0f;
    for (int64_t s0 = (int64_t)blockIdx.x * SB; s0 < n; s0 += (int64_t)gridDim.x * SB) {
        const int ns = (int)min((int64_t)SB, n - s0);
        forward_block(M, L, feat, s0, ns);
        if (tid < SB) {
            float d = 0.0f;
            if (tid < ns) {
                const float e = L.y[tid] - label[s0 + tid];
                sq += e * e;
                d = (2.0f * inv_n) * e;
            }
            L.dy[tid] = d;                       // rows past the end carry no error
        }
        __syncthreads();
        if (tid < MLP_H) {                       // output layer
            const int h = tid;
            float a = 0.0f;
            for (int s = 0; s < SB; ++s) a += bf2f(L.H2[s * LD + h]) * L.dy[s];
            gw3 += a;
        }
        if (tid == 64)
            for (int s = 0; s < SB; ++s) gb3 += L.dy[s];
        __syncthreads();
        // error of layer 2 (bfloat16, in place of H2): dy w3 where the unit was active
        for (int i = tid; i < SB * MLP_H; i += 256) {
            const int s = i / MLP_H, h = i % MLP_H;
            const uint16_t hv = L.H2[s * LD + h];
            L.H2[s * LD + h] = (bf2f(hv) > 0.0f) ? f2bf(L.dy[s] * L.w3[h]) : (uint16_t)0;
        }
        __syncthreads();
        if (tid < MLP_H)
            for (int s = 0; s < SB; ++s) gb2 += bf2f(L.H2[s * LD + tid]);
        // dW2 += H1^T G2 (rows: input units of this wavefront's band)
        for (int nt = 0; nt < 4; ++nt) gW2[nt] = mma_tile(L.H1, 1, LD, L.H2, LD, 1, 16 * w, 16 * nt, SB, gW2[nt]);
        // error reaching layer 1: G2 W2^T (samples of this wavefront's band)
        f32x4 d1[4];
        for (int nt = 0; nt < 4; ++nt) {
            d1[nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
            d1[nt] = mma_tile(L.H2, LD, 1, L.W2, 1, LD, 16 * w, 16 * nt, MLP_H, d1[nt]);
        }
        __syncthreads();                         // every read of H1 for dW2 is done
        for (int nt = 0; nt < 4; ++nt) {
            const int h = 16 * nt + r;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int s = 16 * w + 4 * g + e;
                const uint16_t hv = L.H1[s * LD + h];
                L.H1[s * LD + h] = (bf2f(hv) > 0.0f) ? f2bf(d1[nt][e]) : (uint16_t)0;
            }
        }
        __syncthreads();
        if (tid < MLP_H)
            for (int s = 0; s < SB; ++s) gb1 += bf2f(L.H1[s * LD + tid]);
        // dW1 += X^T G1
        for (int nt = 0; nt < 4; ++nt) gW1[nt] = mma_tile(L.X, 1, LD, L.H1, LD, 1, 16 * w, 16 * nt, SB, gW1[nt]);
        __syncthreads();
    }
    float *out = part + (size_t)blockIdx.x * MLP_PP;
    for (int nt = 0; nt < 4; ++nt) {
        const int c = 16 * nt + r;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = 16 * w + 4 * g + e;
            if (row < MLP_IN) out[MLP_OFF_W1 + row * MLP_H + c] = gW1[nt][e];
            out[MLP_OFF_W2 + row * MLP_H + c] = gW2[nt][e];
        }
    }
    if (tid < MLP_H) {
        out[MLP_OFF_B1 + tid] = gb1;
        out[MLP_OFF_B2 + tid] = gb2;
        out[MLP_OFF_W3 + tid] = gw3;
    }
    if (tid == 64) out[MLP_OFF_B3] = gb3;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) sq += __shfl_xor(sq, o, WAVE);
    if (lane == 0) L.red[w] = sq;
    __syncthreads();
    if (tid == 0) out[MLP_P] = (L.red[0] + L.red[1]) + (L.red[2] + L.red[3]);
}

// grad[p] = sum over workgroups of part[wg][p], in workgroup order (float64), p < MLP_P + 1.
// Sum of the workgroups' partial gradients in float64: a block serves 32 parameters with 8 slices
// of the workgroups each (coalesced rows of 32 partials), the slices then added in slice order, so
// the result does not depend on scheduling.
constexpr int RED_PARAMS = 32, RED_SLICES = 8;

__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float *part, int nwg, float *grad)
{
    __shared__ double acc_s[RED_SLICES][RED_PARAMS];
    const int pl = threadIdx.x % RED_PARAMS, sl = threadIdx.x / RED_PARAMS;
    const int p = blockIdx.x * RED_PARAMS + pl;
    const int per = (nwg + RED_SLICES - 1) / RED_SLICES;
    const int b0 = sl * per, b1 = min(nwg, b0 + per);
    double acc = 0.0;
    if (p <= MLP_P)
        for (int b = b0; b < b1; ++b) acc += (double)part[(size_t)b * MLP_PP + p];
    acc_s[sl][pl] = acc;
    __syncthreads();
    if (sl == 0 && p <= MLP_P) {
        double t = 0.0;
#pragma unroll
        for (int k = 0; k < RED_SLICES; ++k) t += acc_s[k][pl];
        grad[p] = (float)t;
    }
}

__device__ __forceinline__ void refresh_bf16(const MlpView &M, int p)
{
    if (p < MLP_OFF_B1) M.w1b[p] = f2bf(M.theta[p]);
    else if (p >= MLP_OFF_W2 && p < MLP_OFF_B2) M.w2b[p - MLP_OFF_W2] = f2bf(M.theta[p]);
    else if (p >= MLP_OFF_W3 && p < MLP_OFF_B3) M.w3b[p - MLP_OFF_W3] = f2bf(M.theta[p]);
}

// Adam (Kingma and Ba 2015) on the float32 master parameters; moments in float64.
__global__ __launch_bounds__(256) void mlp_adam_kernel(MlpView M, const float *grad, double lr, double beta1,
                                                       double beta2, double eps)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= MLP_P) return;
    const double t = (double)(*M.step + 1);
    const double gr = (double)grad[p];
    const double m = beta1 * M.m[p] + (1.0 - beta1) * gr;
    const double v = beta2 * M.v[p] + (1.0 - beta2) * gr * gr;
    M.m[p] = m;
    M.v[p] = v;
    const double mh = m / (1.0 - pow(beta1, t));
    const double vh = v / (1.0 - pow(beta2, t));
    M.theta[p] = (float)((double)M.theta[p] - lr * mh / (sqrt(vh) + eps));
    refresh_bf16(M, p);
}

__global__ void mlp_step_kernel(MlpView M)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *M.step += 1;
}

__global__ __launch_bounds__(256) void mlp_set_kernel(MlpView M, const float *theta)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < MLP_INP * MLP_H) M.w1b[p] = 0;              // padding rows of W1 stay zero
    if (p < MLP_P) {
        M.theta[p] = theta[p];
        M.m[p] = 0.0;
        M.v[p] = 0.0;
    }
    if (p == 0) *M.step = 0;
}

__global__ __launch_bounds__(256) void mlp_refresh_kernel(MlpView M)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < MLP_P) refresh_bf16(M, p);
}

void launch_mlp_set(const MlpView &M, const float *theta, hipStream_t s)
{
    const int nb = (int)cdiv(MLP_INP * MLP_H > MLP_P ? MLP_INP * MLP_H : MLP_P, 256);
    mlp_set_kernel<<<nb, 256, 0, s>>>(M, theta);
    mlp_refresh_kernel<<<(int)cdiv(MLP_P, 256), 256, 0, s>>>(M);
}

int mlp_grid(int64_t n)
{
    const int64_t b = cdiv(n, SB);
    return (int)(b < MLP_MAX_WG ? b : MLP_MAX_WG);
}

void launch_mlp_forward(const MlpView &M, const uint16_t *feat, int64_t n, float *y, hipStream_t s)
{
    if (n <= 0) return;
    mlp_forward_kernel<<<mlp_grid(n), 256, 0, s>>>(M, feat, n, y);
}

void launch_mlp_grad(const MlpView &M, const uint16_t *feat, const float *label, int64_t n, float *part, float *grad,
                     hipStream_t s)
{
    const int nwg = mlp_grid(n);
    mlp_grad_kernel<<<nwg, 256, 0, s>>>(M, feat, label, n, 1.0f / (float)n, part);
    mlp_reduce_kernel<<<(int)cdiv(MLP_P + 1, RED_PARAMS), 256, 0, s>>>(part, nwg, grad);
}

void launch_mlp_adam(const MlpView &M, const float *grad, float lr, hipStream_t s)
{
    mlp_adam_kernel<<<(int)cdiv(MLP_P, 256), 256, 0, s>>>(M, grad, (double)lr, 0.9, 0.999, 1e-8);
    mlp_step_kernel<<<1, 64, 0, s>>>(M);
}

// ------------------------------------------------------------------------------------------------
// features: light vertices of this batch in 8 equi-areal rings at radii r1 / 2^s, s = 0..3, around
// every hit point (over its grid stencil at radius r1), then the encoded
// network inputs: log1p(count) / 8, the normal and the iteration code, in bfloat16, original order.
// ------------------------------------------------------------------------------------------------

// One wavefront per hit point: the lanes stride through each stencil row together (coalesced
// 16-byte loads) and count into the wavefront's 32 counters in LDS.
constexpr int FEAT_WAVES = 4;

__global__ __launch_bounds__(64 * FEAT_WAVES) void features_kernel(StateView st, int64_t H, const uint32_t *cstart,
                                                                   const float4 *pay, int rec, int nrm_test,
                                                                   float cos_min, float it_code, uint16_t *feat,
                                                                   uint32_t *counts)
{
    __shared__ uint32_t cnt[FEAT_WAVES][32];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t q = (int64_t)blockIdx.x * FEAT_WAVES + wv;
    if (lane < 32) cnt[wv][lane] = 0u;
    __syncthreads();
    if (q < H) {
        const SetHeader *hdr = st.hdr;
        const float p[3] = {st.pos[0][q], st.pos[1][q], st.pos[2][q]};
        const float nv[3] = {st.nrm[0][q], st.nrm[1][q], st.nrm[2][q]};
        const float r1 = hdr->r1;
        float R2[4], T[4][8];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const float R = r1 * (1.0f / (float)(1 << s));
            R2[s] = R * R;
#pragma unroll
            for (int k = 1; k < 8; ++k) T[s][k] = R2[s] * (0.125f * (float)k);
        }
        int c0[3], c1[3];
        if (stencil(hdr, p, r1, c0, c1)) {
            const uint32_t dimx = (uint32_t)hdr->dims[0], dimy = (uint32_t)hdr->dims[1];
            for (int cz = c0[2]; cz <= c1[2]; ++cz)
                for (int cy = c0[1]; cy <= c1[1]; ++cy) {
                    const uint32_t cell = ((uint32_t)cz * dimy + (uint32_t)cy) * dimx;
                    const uint32_t b0 = cstart[cell + (uint32_t)c0[0]], b1 = cstart[cell + (uint32_t)c1[0] + 1u];
                    for (uint32_t j = b0 + (uint32_t)lane; j < b1; j += 64u) {
                        const float4 a = pay[(int64_t)j * rec];
                        const float dx = p[0] - a.x, dy = p[1] - a.y, dz = p[2] - a.z;
                        const float d2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                        if (!(d2 < R2[0])) continue;
                        if (nrm_test) {
                            const float4 bn = pay[(int64_t)j * rec + 2];
                            const float cs = fmaf(nv[2], bn.z, fmaf(nv[1], bn.y, nv[0] * bn.x));
                            if (!(cs >= cos_min)) continue;
                        }
#pragma unroll
                        for (int s = 0; s < 4; ++s) {
                            if (d2 < R2[s]) {
                                int b = 0;
#pragma unroll
                                for (int k = 1; k < 8; ++k) b += (d2 >= T[s][k]) ? 1 : 0;
                                atomicAdd(&cnt[wv][8 * s + b], 1u);
                            }
                        }
                    }
                }
        }
    }
    __syncthreads();
    if (q < H && lane < MLP_IN) {
        const uint32_t o = st.orig[q];
        uint16_t *f = feat + (size_t)o * MLP_IN;
        float v;
        if (lane < 32) {
            const uint32_t c = cnt[wv][lane];
            if (counts) counts[(size_t)o * 32 + lane] = c;
            v = log1pf((float)c) * 0.125f;
        } else {
            v = (lane < 35) ? st.nrm[lane - 32][q] : it_code;
        }
        f[lane] = f2bf(v);
    }
}

void launch_features(const StateView &st, int64_t H, const uint32_t *cstart, const float4 *pay, int rec,
                     bool nrm_test, float cos_min, float it_code, uint16_t *feat, uint32_t *counts, hipStream_t s)
{
    features_kernel<<<(int)cdiv(H, FEAT_WAVES), 64 * FEAT_WAVES, 0, s>>>(st, H, cstart, pay, rec, nrm_test ? 1 : 0,
                                                                         cos_min, it_code, feat, counts);
}

// ------------------------------------------------------------------------------------------------
// proposal: r = clamp(r1 exp(y + margin), lb_{i+1}, r) for the next iteration i + 1; kernels whose radius
// changes drop their retained statistics (they belong to the old disk). The radius histogram for
// the next plan is rebuilt.
// ------------------------------------------------------------------------------------------------

__global__ void zero_hist_kernel(SetHeader *hdr)
{
    if (threadIdx.x < RHIST_BINS) hdr->rhist[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(256) void propose_kernel(StateView st, int64_t H, const float *y, float margin)
{
    __shared__ uint32_t hist[RHIST_BINS];
    if (threadIdx.x < RHIST_BINS) hist[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const float r1 = st.hdr->r1;
    if (q < H) {
        const float lb = st.lbtab[st.hdr->iter + 1];
        const float rc = st.r[q];
        const float rp = fminf(fmaxf(r1 * expf(y[st.orig[q]] + margin), lb), rc);
        if (rp != rc) {
            st.r[q] = rp;
            st.t[q] = 0u;
            st.nseen[q] = 0u;
            for (int i = 0; i < NG * st.nch; ++i)
                st.sq2[(size_t)q * (NG * st.nch) + i] = make_double2(0.0, 0.0);
        }
        atomicAdd(&hist[radius_bin(rp, r1)], 1u);
    }
    __syncthreads();
    if (threadIdx.x < RHIST_BINS && hist[threadIdx.x]) atomicAdd(&st.hdr->rhist[threadIdx.x], hist[threadIdx.x]);
}

void launch_propose(const StateView &st, int64_t H, const float *y, float margin, hipStream_t s)
{
    zero_hist_kernel<<<1, 64, 0, s>>>(st.hdr);
    propose_kernel<<<(int)cdiv(H, 256), 256, 0, s>>>(st, H, y, margin);
}

}  // namespace hk

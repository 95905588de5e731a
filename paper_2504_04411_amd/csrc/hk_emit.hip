// Light-vertex generation for the box scene, on the device: the light pass that feeds the
// estimator (the light sub-paths of Sec. 4's vertex merging, here one segment from an isotropic
// point light to the first wall of a unit box open at z = 1, with an opaque sphere inside).
//
// The generator is counter-based, so a slot depends only on (seed, set, iteration, slot) and the
// iteration index is read from the set's device-resident header: a captured graph of emission plus
// estimator iteration advances by itself on every replay.
//
//   random numbers  Philox4x32-10 (Salmon et al., SC 2011), counter (j, i, s, b), key (seed lo, seed
//                   hi); u = (x >> 8) 2^-24
//   direction       Marsaglia's rejection from the square: block b gives attempts 2b and 2b + 1;
//                   (a, c) = 2u - 1, q = a a + c c, accept 0 < q < 1, d = (a f, c f, 1 - 2q) with
//                   f = 2 sqrt(1 - q); 16 failed attempts leave the slot empty
//   first hit       per-axis exit distances of the unit box, smallest wins (x, then y, then z on
//                   ties); z with d_z > 0 escapes through the open top; the sphere occludes when
//                   its near intersection lies in (0, t)
//
// Every float32 operation is a single correctly rounded IEEE operation (the library is built
// without contraction, division and square root are the correctly rounded ones), so the slots are
// bit-identical to any implementation of the same definition. One thread per slot; the nine output
// arrays are written with coalesced stores (36 bytes per slot, the kernel's only HBM traffic).

#include <math.h>
#include <stdint.h>

#include "hk_internal.h"
#include "hk_kernels.h"

namespace hk {

constexpr int EMIT_THREADS = 256;
constexpr float FOUR_PI_F = 12.566370614359172f;
constexpr int EMIT_BLOCKS = 8;      // Philox blocks per slot: 16 direction attempts

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

__device__ __forceinline__ float unit_u(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }

// One rejection attempt from two words; true when (a, c) lies strictly inside the unit disk.
__device__ __forceinline__ bool attempt(uint32_t x0, uint32_t x1, float &a, float &c, float &q)
{
    const float aa = 2.0f * unit_u(x0) - 1.0f;
    const float cc = 2.0f * unit_u(x1) - 1.0f;
    const float qq = aa * aa + cc * cc;
    if (qq > 0.0f && qq < 1.0f) {
        a = aa;
        c = cc;
        q = qq;
        return true;
    }
    return false;
}

__global__ __launch_bounds__(EMIT_THREADS) void emit_box_kernel(EmitLaunch e)
{
    const int64_t j = (int64_t)blockIdx.x * EMIT_THREADS + threadIdx.x;
    if (j >= e.J) return;
    const uint32_t it = (uint32_t)e.hdr->iter;     // iterations started so far = this iteration's index

    float a = 0.0f, c = 0.0f, q = 0.0f;
    bool drawn = false;
    for (int b = 0; b < EMIT_BLOCKS && !drawn; ++b) {
        const uint4 x = philox4x32_10(make_uint4((uint32_t)j, it, e.set_id, (uint32_t)b), e.key0, e.key1);
        drawn = attempt(x.x, x.y, a, c, q) || attempt(x.z, x.w, a, c, q);
    }
    const float f = 2.0f * __builtin_sqrtf(1.0f - q);
    const float d[3] = {a * f, c * f, 1.0f - 2.0f * q};

    float tx[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        const float L = e.L[ax];
        tx[ax] = d[ax] > 0.0f ? (1.0f - L) / d[ax] : d[ax] < 0.0f ? (0.0f - L) / d[ax] : INFINITY;
    }
    const float t = fminf(fminf(tx[0], tx[1]), tx[2]);
    const int hit = tx[0] == t ? 0 : tx[1] == t ? 1 : 2;
    const bool escaped = hit == 2 && d[2] > 0.0f;

    const float ox = e.L[0] - e.C[0], oy = e.L[1] - e.C[1], oz = e.L[2] - e.C[2];
    const float B = (d[0] * ox + d[1] * oy) + d[2] * oz;
    const float Q = ((ox * ox + oy * oy) + oz * oz) - e.R * e.R;
    const float D = B * B - Q;
    const float ts = -B - __builtin_sqrtf(fmaxf(D, 0.0f));
    const bool occluded = D > 0.0f && ts > 0.0f && ts < t;
    const bool keep = drawn && !escaped && !occluded;

#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
        float p = fminf(fmaxf(e.L[ax] + t * d[ax], 0.0f), 1.0f);
        float n = 0.0f;
        if (hit == ax) {
            p = d[ax] > 0.0f ? 1.0f : 0.0f;
            n = d[ax] > 0.0f ? -1.0f : 1.0f;
        }
        e.pos[ax][j] = keep ? p : __builtin_nanf("");
        e.nrm[ax][j] = keep ? n : 0.0f;
        e.flux[ax][j] = keep ? e.power : 0.0f;
    }
    if (e.mis[0]) {
        // reciprocal of the area density of the vertex: isotropic emission 1 / (4 pi) times
        // cos / t^2, the cosine being the direction's component on the hit axis
        const float dh = fabsf(hit == 0 ? d[0] : hit == 1 ? d[1] : d[2]);
        const float dvcm = (FOUR_PI_F * (t * t)) / dh;
        e.mis[0][j] = keep ? dvcm : 0.0f;
        e.mis[1][j] = 0.0f;
        e.mis[2][j] = 0.0f;
    }
}

// Next-event connection of camera vertex q to the point light (the VC technique of the VCM
// estimator for the box scene) with the balance-heuristic weight against merging:
//   w_VC = 1 / (1 + eta p_L(x)),  eta = J pi r^2,  p_L(x) = cos / (4 pi d^2),
// adding w_VC beta_C I cos V / d^2 to the iteration's flux-density estimate (compensated pairs).
// The shadow test is float32 in the stated operation order; the radius is the one this iteration
// merges with (the kernel runs before the gather of the iteration).
__global__ __launch_bounds__(256) void connect_box_kernel(ConnectLaunch c)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= c.H) return;
    const StateView &st = c.st;
    const float px = st.pos[0][q], py = st.pos[1][q], pz = st.pos[2][q];
    const float nx = st.nrm[0][q], ny = st.nrm[1][q], nz = st.nrm[2][q];
    const float r = st.r[q];
    // shadow test of the segment x -> light
    const float wx = c.L[0] - px, wy = c.L[1] - py, wz = c.L[2] - pz;
    const float d2 = (wx * wx + wy * wy) + wz * wz;
    const float dist = __builtin_sqrtf(d2);
    const float ux = wx / dist, uy = wy / dist, uz = wz / dist;
    const float ox = px - c.C[0], oy = py - c.C[1], oz = pz - c.C[2];
    const float B = (ux * ox + uy * oy) + uz * oz;
    const float Q = ((ox * ox + oy * oy) + oz * oz) - c.R * c.R;
    const float D = B * B - Q;
    const float t0 = -B - __builtin_sqrtf(fmaxf(D, 0.0f));
    const bool blocked = D > 0.0f && t0 > 0.0f && t0 < dist;
    const float cs = fmaxf(0.0f, (ux * nx + uy * ny) + uz * nz);
    const float eta = c.Jf * (PI_F * (r * r));
    const float pl = cs / (FOUR_PI_F * d2);
    const float w = 1.0f / (1.0f + eta * pl);
    const float e = blocked ? 0.0f : ((w * c.intensity) * cs) / d2;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float *ts = st.tau0 + (size_t)(2 * ch) * st.astride;
        float *tc = st.tau0 + (size_t)(2 * ch + 1) * st.astride;
        float sv = ts[q], cv = tc[q];
        acc2(sv, cv, st.cb[ch][q] * e);
        ts[q] = sv;
        tc[q] = cv;
    }
}

void launch_connect_box(const ConnectLaunch &c, hipStream_t s)
{
    if (c.H <= 0) return;
    connect_box_kernel<<<(int)cdiv(c.H, 256), 256, 0, s>>>(c);
}

void launch_emit_box(const EmitLaunch &e, hipStream_t s)
{
    if (e.J <= 0) return;
    emit_box_kernel<<<(int)cdiv(e.J, EMIT_THREADS), EMIT_THREADS, 0, s>>>(e);
}

}  // namespace hk

// Gain-applied visibilities and their adjoint with respect to the complex gains.
//
// Per-input complex gains (station, polarisation, subband, channel) are constant over a
// block, so applying them to the channelised samples before the X stage equals scaling each
// stored visibility:  V'_ab = g_a conj(g_b) V0_ab.  For a real loss with upstream gradient
// G = dL/dRe V' + i dL/dIm V', the gradient with respect to g_k (same convention) is
//     sum_{entries with b = k} conj(G_ab) g_a V0_ab + sum_{entries with a = k} G_ab g_b conj(V0_ab).
// Both kernels read the visibilities once per use and are bandwidth-bound; the adjoint gives
// each input of a channel to one thread and sums its entries in a fixed order (no atomics,
// bit-reproducible).
#include "cobalt_internal.h"

namespace cobalt {
namespace {

__device__ __forceinline__ float2 cmul(float2 x, float2 y) {
    return make_float2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x);
}
__device__ __forceinline__ float2 cconj(float2 x) { return make_float2(x.x, -x.y); }

__global__ __launch_bounds__(256) void apply_gains_kernel(const float2* __restrict__ vis0, const float2* __restrict__ gains,
                                                          float2* __restrict__ vis, int64_t n_entries, int B, int M) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n_entries) return;
    const int q = (int)(e & 3);
    const int64_t rest = e >> 2;
    const int bl = (int)(rest % B);
    const int64_t ch = rest / B;
    int s1 = (int)((sqrtf(8.f * bl + 1.f) - 1.f) * 0.5f);
    while (s1 * (s1 + 1) / 2 > bl) --s1;
    while ((s1 + 1) * (s1 + 2) / 2 <= bl) ++s1;
    const int s2 = bl - s1 * (s1 + 1) / 2;
    const float2 ga = gains[ch * M + 2 * s1 + (q >> 1)];
    const float2 gb = gains[ch * M + 2 * s2 + (q & 1)];
    vis[e] = cmul(cmul(ga, cconj(gb)), vis0[e]);
}

__global__ __launch_bounds__(256) void apply_gains_adjoint_kernel(const float2* __restrict__ vis0, const float2* __restrict__ gains,
                                                                  const float2* __restrict__ grad_vis, float2* __restrict__ grad_gains,
                                                                  int S, int M) {
    const int k = threadIdx.x;
    if (k >= M) return;
    const int64_t ch = blockIdx.x;
    const int64_t B = (int64_t)S * (S + 1) / 2;
    const float2* v0 = vis0 + ch * B * 4;
    const float2* G = grad_vis + ch * B * 4;
    const float2* g = gains + ch * M;
    const int sk = k >> 1, pk = k & 1;
    float2 acc = make_float2(0.f, 0.f);
    // entries with a = k: baselines (sk, s2), s2 <= sk, pol pair (pk, p2)
    for (int s2 = 0; s2 <= sk; ++s2) {
        const int64_t base = ((int64_t)sk * (sk + 1) / 2 + s2) * 4 + 2 * pk;
#pragma unroll
        for (int p2 = 0; p2 < 2; ++p2) {
            const float2 t = cmul(cmul(G[base + p2], g[2 * s2 + p2]), cconj(v0[base + p2]));
            acc.x += t.x;
            acc.y += t.y;
        }
    }
    // entries with b = k: baselines (s1, sk), s1 >= sk, pol pair (p1, pk)
    for (int s1 = sk; s1 < S; ++s1) {
        const int64_t base = ((int64_t)s1 * (s1 + 1) / 2 + sk) * 4 + pk;
#pragma unroll
        for (int p1 = 0; p1 < 2; ++p1) {
            const float2 t = cmul(cmul(cconj(G[base + 2 * p1]), g[2 * s1 + p1]), v0[base + 2 * p1]);
            acc.x += t.x;
            acc.y += t.y;
        }
    }
    grad_gains[ch * M + k] = acc;
}

}  // namespace

hipError_t launch_apply_gains(const void* vis0, const void* gains, void* vis, int n_chan, int S, hipStream_t st) {
    const int64_t B = (int64_t)S * (S + 1) / 2;
    const int64_t n = (int64_t)n_chan * B * 4;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(apply_gains_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (const float2*)vis0,
                       (const float2*)gains, (float2*)vis, n, (int)B, 2 * S);
    return hipGetLastError();
}

hipError_t launch_apply_gains_adjoint(const void* vis0, const void* gains, const void* grad_vis, void* grad_gains, int n_chan,
                                      int S, hipStream_t st) {
    if (n_chan == 0) return hipSuccess;
    hipLaunchKernelGGL(apply_gains_adjoint_kernel, dim3((unsigned)n_chan), dim3(256), 0, st, (const float2*)vis0,
                       (const float2*)gains, (const float2*)grad_vis, (float2*)grad_gains, S, 2 * S);
    return hipGetLastError();
}

}  // namespace cobalt

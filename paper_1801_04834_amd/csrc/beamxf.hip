// Output-resolution transform of beamformed voltages ("Signal processing with GPU kernels",
// sec. 7.5: beams are formed at 256 channels per subband and then transformed to the requested
// output resolution, often 1 or 16 channels per subband; "System requirements", sec. 5: time
// resolution is traded for frequency resolution within a subband).
//
// Per subband, beam and polarisation, the 256 channel values of each channel sample j go back
// to 256 time samples with an inverse DFT (scaled 1/C; channel c carries frequency index
// c - C/2), the rows form one time series at the subband rate, and every group of C_out
// consecutive samples gets an unnormalised forward C_out-point DFT (output channel c' carries
// index c' - C_out/2).  Optionally Stokes parameters of the transformed voltages, summed over
// n_int consecutive output samples of a row.
//
// Work decomposition: one workgroup of 512 threads per (subband, channel sample, group of 16
// beams) = 32 transforms (2 polarisations x 16 beams), 16 threads per transform.  The 256-point
// inverse DFT runs as 16 x 16 (c = c1 + 16 c2, n = 16 n1 + n2):
//     u[16 n1 + n2] = (1/C) (-1)^n sum_c1 w16^(n1 c1) w256^(n2 c1) sum_c2 B[c1 + 16 c2] w16^(n2 c2)
// (w_N = exp(+2 pi i / N)); pass 1 (thread c1) and pass 2 (thread n2) are in-register 16-point
// transforms, exchanged through one LDS array; pass 3 (thread d) forward-transforms the groups
// of its 16 consecutive samples.  The outputs leave from LDS with the beams fastest (128-byte
// rows per polarisation).  Memory-bound: one read of the voltages, one write of the outputs.
#include "cobalt_internal.h"

namespace cobalt {
namespace {

constexpr int kXC = 256;                 // input channels (the beamformer's front end)
constexpr int kBG = 16;                  // beams per workgroup
constexpr int kNF = 2 * kBG;             // transforms per workgroup
constexpr int kLd = kNF + 1;             // LDS row stride in float2 (one pad element)
constexpr int kXThreads = 16 * kNF;      // 512

constexpr double kPiX = 3.141592653589793238462643383279502884;
constexpr double xt_sin(double x) {
    double term = x, sum = x;
    for (int n = 1; n < 24; ++n) { term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0)); sum += term; }
    return sum;
}
constexpr double xt_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 24; ++n) { term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n)); sum += term; }
    return sum;
}
// cos and sin of 2 pi k / N rounded to float (reduced to the first octant's quadrant first)
constexpr float cos2pi(int k, int N) {
    k = ((k % N) + N) % N;
    const int q = (4 * k) / N, r = 4 * k - q * N;          // angle = (q + r/N) * pi/2
    const double th = kPiX * r / (2.0 * N), c = xt_cos(th), s = xt_sin(th);
    return (float)(q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s);
}
constexpr float sin2pi(int k, int N) {
    k = ((k % N) + N) % N;
    const int q = (4 * k) / N, r = 4 * k - q * N;
    const double th = kPiX * r / (2.0 * N), c = xt_cos(th), s = xt_sin(th);
    return (float)(q == 0 ? s : q == 1 ? c : q == 2 ? -s : -c);
}

template <int N>
constexpr int bitrev(int i) {
    int r = 0;
    for (int b = 1; b < N; b <<= 1) {
        r <<= 1;
        if (i & b) r |= 1;
    }
    return r;
}

// One radix-2 decimation-in-frequency stage (half-span SP) of an N-point transform with
// kernel exp(SIGN 2 pi i n k / N); the k-th butterfly of a group multiplies the difference by
// exp(SIGN 2 pi i k / (2 SP)).
template <int N, int SIGN, int SP>
__device__ __forceinline__ void dif_pass(float (&re)[N], float (&im)[N]) {
#pragma unroll
    for (int start = 0; start < N; start += 2 * SP) {
#pragma unroll
        for (int k = 0; k < SP; ++k) {
            const int i0 = start + k, i1 = i0 + SP;
            const float ar = re[i0], ai = im[i0], br = re[i1], bi = im[i1];
            re[i0] = ar + br;
            im[i0] = ai + bi;
            const float dr = ar - br, di = ai - bi;
            const float c = cos2pi(k, 2 * SP), s = SIGN * sin2pi(k, 2 * SP);
            if (k == 0) {
                re[i1] = dr;
                im[i1] = di;
            } else {
                re[i1] = dr * c - di * s;
                im[i1] = dr * s + di * c;
            }
        }
    }
}
// N-point transform in registers, natural-order input; element i holds bin bitrev<N>(i).
template <int N, int SIGN>
__device__ __forceinline__ void dft(float (&re)[N], float (&im)[N]) {
    if constexpr (N >= 2) dif_pass<N, SIGN, N / 2>(re, im);
    if constexpr (N >= 4) dif_pass<N, SIGN, N / 4>(re, im);
    if constexpr (N >= 8) dif_pass<N, SIGN, N / 8>(re, im);
    if constexpr (N >= 16) dif_pass<N, SIGN, N / 16>(re, im);
    static_assert(N <= 16, "transforms of up to 16 points in registers");
}

template <int COUT, int NS>
__global__ __launch_bounds__(kXThreads) void beam_transform_kernel(TfArgs a) {
    __shared__ float2 buf[kXC * kLd];
    const int tid = threadIdx.x;
    const int f = tid >> 4, d = tid & 15;                   // transform f = p kBG + b, digit d
    const int bg = (int)(blockIdx.x % (unsigned)a.n_bg);
    const int rest = (int)(blockIdx.x / (unsigned)a.n_bg);
    const int j = rest % a.n_c, sb = rest / a.n_c;
    const int b0 = bg * kBG;
    const int64_t row2 = 2 * (int64_t)a.NB;                 // float2 per (channel, sample) row

    // ---- load the 256 channels x 32 transforms: buf[c][f] ----
    const float2* __restrict__ vin = (const float2*)a.vin + ((int64_t)sb * kXC * a.n_c + j) * row2;
#pragma unroll 4
    for (int i = 0; i < kXC * kNF / kXThreads; ++i) {
        const int e = tid + kXThreads * i, c = e >> 5, ff = e & 31, p = ff >> 4, bb = ff & 15;
        float2 v = make_float2(0.f, 0.f);
        if (b0 + bb < a.NB) v = vin[(int64_t)c * a.n_c * row2 + p * a.NB + b0 + bb];
        buf[c * kLd + ff] = v;
    }
    __syncthreads();

    float xr[16], xi[16];
    // ---- pass 1 (c1 = d): inverse 16-point DFT over c2 of B[c1 + 16 c2], then w256^(n2 c1) ----
#pragma unroll
    for (int c2 = 0; c2 < 16; ++c2) {
        const float2 v = buf[(d + 16 * c2) * kLd + f];
        xr[c2] = v.x;
        xi[c2] = v.y;
    }
    dft<16, +1>(xr, xi);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int n2 = bitrev<16>(i);
        float s, c;
        sincospif((float)(2 * n2 * d) / (float)kXC, &s, &c);
        buf[(d * 16 + n2) * kLd + f] = make_float2(xr[i] * c - xi[i] * s, xr[i] * s + xi[i] * c);
    }
    __syncthreads();
    // ---- pass 2 (n2 = d): inverse 16-point DFT over c1; time sample n = 16 n1 + n2 ----
#pragma unroll
    for (int c1 = 0; c1 < 16; ++c1) {
        const float2 v = buf[(c1 * 16 + d) * kLd + f];
        xr[c1] = v.x;
        xi[c1] = v.y;
    }
    dft<16, +1>(xr, xi);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int n = 16 * bitrev<16>(i) + d;
        const float sc = (n & 1) ? -1.f / kXC : 1.f / kXC;   // (-1)^n from index c - C/2, and 1/C
        buf[n * kLd + f] = make_float2(xr[i] * sc, xi[i] * sc);
    }
    __syncthreads();
    // ---- pass 3 (samples 16 d .. 16 d + 15): forward COUT-point DFTs of consecutive groups ----
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const float2 v = buf[(16 * d + k) * kLd + f];
        // (-1)^m: output channel c' carries frequency index c' - COUT/2
        const bool neg = COUT > 1 && (k % COUT) % 2 == 1;
        xr[k] = neg ? -v.x : v.x;
        xi[k] = neg ? -v.y : v.y;
    }
    if constexpr (COUT > 1) {
#pragma unroll
        for (int q = 0; q < 16 / COUT; ++q) {
            float yr[COUT], yi[COUT];
#pragma unroll
            for (int m = 0; m < COUT; ++m) {
                yr[m] = xr[q * COUT + m];
                yi[m] = xi[q * COUT + m];
            }
            dft<COUT, -1>(yr, yi);
#pragma unroll
            for (int i = 0; i < COUT; ++i) {
                xr[q * COUT + bitrev<COUT>(i)] = yr[i];
                xi[q * COUT + bitrev<COUT>(i)] = yi[i];
            }
        }
    }
    // no barrier needed before this write: each thread rewrites exactly the slots it read
#pragma unroll
    for (int k = 0; k < 16; ++k) buf[(16 * d + k) * kLd + f] = make_float2(xr[k], xi[k]);
    __syncthreads();

    // ---- outputs, beams fastest: slot s = g_local COUT + c' of row j ----
    constexpr int kSlots = kXC;                              // g_local in [0, 256/COUT), c' < COUT
    if (a.vout) {
        // [SB][G][COUT][P][NB] with G = N_c 256 / COUT; this row's slots are contiguous
        float2* __restrict__ vo = (float2*)a.vout + ((int64_t)sb * a.n_c + j) * kXC * row2;
        for (int it = tid; it < kSlots * kNF; it += kXThreads) {
            const int ff = it & 31, s = it >> 5, p = ff >> 4;
            if (b0 + (ff & 15) < a.NB) vo[(int64_t)s * row2 + p * a.NB + b0 + (ff & 15)] = buf[s * kLd + ff];
        }
    }
    if constexpr (NS > 0) {
        // [SB][G / n_int][COUT][NS][NB]; a row holds 256 / COUT output samples, n_int divides it
        const int per_row = kXC / COUT / a.n_int;            // Stokes samples per row
        float* __restrict__ so = (float*)a.sout + ((int64_t)sb * a.n_c + j) * per_row * COUT * NS * a.NB;
        for (int it = tid; it < per_row * COUT * kBG; it += kXThreads) {
            const int bb = it & 15, cc = (it >> 4) % COUT, go = (it >> 4) / COUT;
            float acc[4] = {0.f, 0.f, 0.f, 0.f};
            for (int u = 0; u < a.n_int; ++u) {
                const int s = (go * a.n_int + u) * COUT + cc;
                const float2 X = buf[s * kLd + bb], Y = buf[s * kLd + kBG + bb];
                const float xx = X.x * X.x + X.y * X.y, yy = Y.x * Y.x + Y.y * Y.y;
                acc[0] += xx + yy;
                if constexpr (NS == 4) {
                    acc[1] += xx - yy;
                    acc[2] += 2.f * (X.x * Y.x + X.y * Y.y);
                    acc[3] += 2.f * (X.y * Y.x - X.x * Y.y);
                }
            }
            if (b0 + bb < a.NB) {
#pragma unroll
                for (int k = 0; k < NS; ++k) so[((int64_t)(go * COUT + cc) * NS + k) * a.NB + b0 + bb] = acc[k];
            }
        }
    }
}

template <int COUT>
hipError_t launch_cout(const TfArgs& a, hipStream_t st) {
    const dim3 grid((unsigned)((int64_t)a.SB * a.n_c * a.n_bg)), block(kXThreads);
    switch (a.sout ? a.n_stokes : 0) {
        case 0: hipLaunchKernelGGL((beam_transform_kernel<COUT, 0>), grid, block, 0, st, a); break;
        case 1: hipLaunchKernelGGL((beam_transform_kernel<COUT, 1>), grid, block, 0, st, a); break;
        case 4: hipLaunchKernelGGL((beam_transform_kernel<COUT, 4>), grid, block, 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_beam_transform(const TfArgs& a, hipStream_t st) {
    if ((int64_t)a.SB * a.n_c * a.n_bg == 0) return hipSuccess;
    switch (a.c_out) {
        case 1: return launch_cout<1>(a, st);
        case 2: return launch_cout<2>(a, st);
        case 4: return launch_cout<4>(a, st);
        case 8: return launch_cout<8>(a, st);
        case 16: return launch_cout<16>(a, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace cobalt

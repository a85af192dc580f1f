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
// Factoring (C = 256, c = c1 + 16 c2, time n = 16 n1 + n2, n2 = C_out q + m, w_N = e^(2 pi i/N)):
//     u[n]          = (-1)^n / C  sum_c1 w16^(n1 c1) w256^(n2 c1) A[c1, n2],
//     A[c1, n2]     = sum_c2 B[c1 + 16 c2] w16^(n2 c2),
// and the output channel c' of output sample g = Q n1 + q (Q = 16 / C_out) is
//     O[g, c']      = sum_c1 w16^(n1 c1) Z[c1, q, c'],
//     Z[c1, q, c']  = sum_m w_Cout^(-m c') T[c1, n2] A[c1, n2],
//     T[c1, n2]     = w256^(n2 c1) / C, times (-1)^n2 when C_out = 1
// (for even C_out the two half-band signs (-1)^n and (-1)^m cancel).  So one thread per c1
// does the inverse 16-point DFT over c2, the twiddle and the forward C_out-point DFTs over m,
// all in registers; one LDS exchange hands Z to one thread per t = C_out q + c', which does the
// inverse 16-point DFT over c1 and holds the outputs of slots 16 n1 + t of the row.
//
// Work decomposition: one workgroup of 512 threads per (subband, channel sample): 16 digits x
// 32 transforms (2 polarisations x 16 beams, the transform index fastest in a wavefront, so a
// load instruction reads 128-byte runs of beams; rows padded to whole 128-byte lines keep
// every such run on one line).  The workgroup walks the groups of 16 beams of its row, loading
// the next group into registers while it transforms the current one; the twiddles come from a
// 2 KB LDS table.  Stokes parameters at C_out = 16 are summed in registers (the output channel
// is the thread's digit, the polarisations sit 16 lanes apart); at other C_out the outputs go
// through LDS to be summed across threads.  Memory-bound: one read of the voltages, one write
// of the outputs.
#include "cobalt_internal.h"

namespace cobalt {
namespace {

constexpr int kXC = 256;                 // input channels (the beamformer's front end)
constexpr int kBG = 16;                  // beams per group
constexpr int kNF = 2 * kBG;             // transforms per group
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

// w256^k for k < 256 (the pass-1 twiddles, indexed by n2 c1 mod 256)
struct TwTable {
    float re[kXC], im[kXC];
};
constexpr TwTable make_tw() {
    TwTable t{};
    for (int k = 0; k < kXC; ++k) {
        t.re[k] = cos2pi(k, kXC);
        t.im[k] = sin2pi(k, kXC);
    }
    return t;
}
__constant__ TwTable kTw = make_tw();

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
            } else if (4 * k == 2 * SP) {                  // exp(SIGN i pi/2) = SIGN i
                re[i1] = -SIGN * di;
                im[i1] = SIGN * dr;
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
__global__ __launch_bounds__(kXThreads, 4) void beam_transform_kernel(TfArgs a) {
    // exchange rows 16 t + c1 (Z of digit c1 for thread t), later output slots s; 32 transforms
    __shared__ float2 buf[kXC * kNF];
    const int tid = threadIdx.x;
    const int d = tid >> 5, f = tid & 31, p = f >> 4, b = f & 15;
    // blocks are dealt to the 8 XCDs in turn: give each XCD a contiguous run of rows, so that
    // the cache lines two neighbouring rows share are fetched into one L2
    const unsigned nblk = gridDim.x, per = nblk / 8u, rem = nblk % 8u;
    const unsigned xcd = blockIdx.x % 8u, row = xcd * per + min(xcd, rem) + blockIdx.x / 8u;
    const int j = (int)(row % (unsigned)a.n_c), sb = (int)(row / (unsigned)a.n_c);
    const int64_t row2 = 2 * (int64_t)a.vstride;            // float2 per (channel, sample) row

    // pass-1 twiddles w256^k / C in LDS (same address across a half-wavefront: broadcast reads)
    __shared__ float2 tw[kXC];
    if (tid < kXC) tw[tid] = make_float2(kTw.re[tid] * (1.f / kXC), kTw.im[tid] * (1.f / kXC));
    __syncthreads();

    // inputs of digit d: channels d + 16 c2 of row (sb, j), transform f.  Raw buffer loads: the
    // row's base in scalar registers, one 32-bit lane offset, the channel step (c2) and the beam
    // group step in the scalar offset, so the 16 loads cost no address arithmetic per lane
    // (the host keeps a subband's voltages below 4 GiB)
    const int64_t base = ((int64_t)sb * kXC * a.n_c + j) * row2;              // float2
    const uint32_t extent = (uint32_t)(((int64_t)kXC * a.n_c - j) * row2 * 8); // bytes to the subband's end
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc((void*)((const float2*)a.vin + base), (short)0, (int)extent, 0x00020000);
    const uint32_t voff = (uint32_t)((((int64_t)d * a.n_c) * row2 + p * a.vstride) * 8);
    const uint32_t cstep = (uint32_t)(16 * (int64_t)a.n_c * row2 * 8);       // bytes from channel c to c + 16
    // lanes past the last beam read the last beam instead (their results are never stored, and
    // every step before the stores keeps lanes apart, the polarisation swap pairing lanes of one beam)
    auto load = [&](float2 (&nxt)[16], int bg) {
        const uint32_t o = voff + (uint32_t)min(bg * kBG + b, a.NB - 1) * 8u;
#pragma unroll
        for (int c2 = 0; c2 < 16; ++c2) {
            const auto v = __builtin_amdgcn_raw_buffer_load_b64(rsrc, (int)o, (int)(c2 * cstep), 0);
            nxt[c2] = make_float2(__uint_as_float(v[0]), __uint_as_float(v[1]));
        }
    };
    const int64_t rowbase = ((int64_t)sb * a.n_c + j) * kXC;   // first output slot of the row
    const int nint_log2 = __builtin_ctz((unsigned)a.n_int);

    // one beam group: consumes its inputs v
    auto group = [&](float2 (&v)[16], int bg) {
        float xr[16], xi[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            xr[i] = v[i].x;
            xi[i] = v[i].y;
        }
        const bool live = bg * kBG + b < a.NB;

        // ---- digit c1 = d: inverse DFT over c2, twiddle, forward C_out-point DFTs over m ----
        dft<16, +1>(xr, xi);
        // twiddle w256^(n2 c1) / C, and (-1)^n2 when C_out = 1; n2 = 0: 1/C
        xr[0] *= 1.f / kXC;
        xi[0] *= 1.f / kXC;
#pragma unroll
        for (int i = 1; i < 16; ++i) {
            const int n2 = bitrev<16>(i);
            const float2 w = tw[(n2 * d) & (kXC - 1)];
            const float sg = (COUT == 1 && (n2 & 1)) ? -1.f : 1.f;
            const float r = sg * (xr[i] * w.x - xi[i] * w.y);
            xi[i] = sg * (xr[i] * w.y + xi[i] * w.x);
            xr[i] = r;
        }
        __syncthreads();                                    // the previous group's readers are done
        if constexpr (COUT == 1) {
#pragma unroll
            for (int i = 0; i < 16; ++i) buf[(16 * bitrev<16>(i) + d) * kNF + f] = make_float2(xr[i], xi[i]);
        } else {
#pragma unroll
            for (int q = 0; q < 16 / COUT; ++q) {
                float yr[COUT], yi[COUT];
#pragma unroll
                for (int m = 0; m < COUT; ++m) {
                    yr[m] = xr[bitrev<16>(COUT * q + m)];
                    yi[m] = xi[bitrev<16>(COUT * q + m)];
                }
                dft<COUT, -1>(yr, yi);
#pragma unroll
                for (int i = 0; i < COUT; ++i) {
                    const int t = COUT * q + bitrev<COUT>(i);
                    buf[(16 * t + d) * kNF + f] = make_float2(yr[i], yi[i]);
                }
            }
        }
        __syncthreads();

        // ---- thread t = d: inverse DFT over c1; element i holds n1 = bitrev(i), slot 16 n1 + t ----
#pragma unroll
        for (int c1 = 0; c1 < 16; ++c1) {
            const float2 v = buf[(16 * d + c1) * kNF + f];
            xr[c1] = v.x;
            xi[c1] = v.y;
        }
        dft<16, +1>(xr, xi);

        if (a.vout && bg * kBG + b < a.vstride) {              // padding beams of the group get zeros
            // [SB][G][COUT][P][NB] with G = N_c 256 / COUT: slot s of the row is g_local COUT + c';
            // the row's 256 slots through one buffer resource, slot step in the scalar offset
            const __amdgpu_buffer_rsrc_t orsrc = __builtin_amdgcn_make_buffer_rsrc(
                (void*)((float2*)a.vout + rowbase * row2), (short)0, (int)(uint32_t)(kXC * row2 * 8), 0x00020000);
            const uint32_t ooff = (uint32_t)((d * row2 + p * a.vstride + b) * 8);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                __attribute__((ext_vector_type(2))) unsigned v = {live ? __float_as_uint(xr[i]) : 0u,
                                                                   live ? __float_as_uint(xi[i]) : 0u};
                __builtin_amdgcn_raw_buffer_store_b64(v, orsrc, (int)ooff, (int)((16 * bitrev<16>(i) * row2 + bg * kBG) * 8), 0);
            }
        }
        if constexpr (NS > 0 && COUT == 16) {
            // output sample n1 of the row, output channel d; polarisation 1 sits 16 lanes above
            // polarisation 0, and the swap hands every lane both (first: pol 0, second: pol 1)
            float* __restrict__ so = (float*)a.sout + (((int64_t)sb * a.n_c + j) * (16 >> nint_log2) * COUT) * NS * a.NB
                                     + (int64_t)d * NS * a.NB + bg * kBG + b;
            float acc[NS];
#pragma unroll
            for (int k = 0; k < NS; ++k) acc[k] = 0.f;
#pragma unroll
            for (int n1 = 0; n1 < 16; ++n1) {
                const int i = bitrev<16>(n1);
                if constexpr (NS == 1) {
                    acc[0] = fmaf(xr[i], xr[i], acc[0]);
                    acc[0] = fmaf(xi[i], xi[i], acc[0]);
                } else {
                    const auto sr = __builtin_amdgcn_permlane16_swap(__float_as_uint(xr[i]), __float_as_uint(xr[i]), false, false);
                    const auto si = __builtin_amdgcn_permlane16_swap(__float_as_uint(xi[i]), __float_as_uint(xi[i]), false, false);
                    const float Xr = __uint_as_float(sr[0]), Yr = __uint_as_float(sr[1]);
                    const float Xi = __uint_as_float(si[0]), Yi = __uint_as_float(si[1]);
                    const float xx = Xr * Xr + Xi * Xi, yy = Yr * Yr + Yi * Yi;
                    acc[0] += xx + yy;
                    acc[1] += xx - yy;
                    acc[2] += 2.f * (Xr * Yr + Xi * Yi);
                    acc[3] += 2.f * (Xi * Yr - Xr * Yi);
                }
                if (((n1 + 1) & (a.n_int - 1)) == 0) {       // the last sample of a Stokes sample
                    if constexpr (NS == 1) {
                        const auto sw = __builtin_amdgcn_permlane16_swap(__float_as_uint(acc[0]), __float_as_uint(acc[0]), false, false);
                        acc[0] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
                    }
                    if (p == 0 && live) {
                        const int64_t go = n1 >> nint_log2;
#pragma unroll
                        for (int k = 0; k < NS; ++k) so[(go * COUT * NS + k) * a.NB] = acc[k];
                    }
#pragma unroll
                    for (int k = 0; k < NS; ++k) acc[k] = 0.f;
                }
            }
        } else if constexpr (NS > 0) {
            // sums across threads: the outputs go to LDS as slot rows, then one thread per
            // (Stokes sample, output channel, beam) adds its n_int samples
            __syncthreads();                                // every thread has read its Z rows
#pragma unroll
            for (int i = 0; i < 16; ++i) buf[(16 * bitrev<16>(i) + d) * kNF + f] = make_float2(xr[i], xi[i]);
            __syncthreads();
            const int per_row = (kXC / COUT) >> nint_log2;  // Stokes samples per row
            float* __restrict__ so = (float*)a.sout + (((int64_t)sb * a.n_c + j) * per_row * COUT) * NS * a.NB + bg * kBG;
            for (int it = tid; it < per_row * COUT * kBG; it += kXThreads) {
                const int bb = it & 15, cc = (it >> 4) % COUT, go = (it >> 4) / COUT;
                float acc[4] = {0.f, 0.f, 0.f, 0.f};
                for (int u = 0; u < a.n_int; ++u) {
                    const int s = (go * a.n_int + u) * COUT + cc;
                    const float2 X = buf[s * kNF + bb], Y = buf[s * kNF + kBG + bb];
                    const float xx = X.x * X.x + X.y * X.y, yy = Y.x * Y.x + Y.y * Y.y;
                    acc[0] += xx + yy;
                    if constexpr (NS == 4) {
                        acc[1] += xx - yy;
                        acc[2] += 2.f * (X.x * Y.x + X.y * Y.y);
                        acc[3] += 2.f * (X.y * Y.x - X.x * Y.y);
                    }
                }
                if (bg * kBG + bb < a.NB) {
#pragma unroll
                    for (int k = 0; k < NS; ++k) so[((int64_t)(go * COUT + cc) * NS + k) * a.NB + bb] = acc[k];
                }
            }
        }
    };

    // the next group's loads are in flight while a group is transformed
    float2 nxt[16];
    load(nxt, 0);
    for (int bg = 0; bg < a.n_bg; ++bg) {
        float2 cur[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) cur[i] = nxt[i];
        if (bg + 1 < a.n_bg) load(nxt, bg + 1);
        group(cur, bg);
    }
}

template <int COUT>
hipError_t launch_cout(const TfArgs& a, hipStream_t st) {
    const dim3 grid((unsigned)((int64_t)a.SB * a.n_c)), block(kXThreads);
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
    if (a.n_int <= 0 || (a.n_int & (a.n_int - 1)) != 0 || a.n_int > kXC / a.c_out) return hipErrorInvalidValue;
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

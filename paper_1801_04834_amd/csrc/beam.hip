// Beamformer on the channelised data ("Signal processing with GPU kernels", sec. 7.5;
// "System requirements", sec. 5): coherent beams shift every station's channel by a per-beam
// phase and sum over stations; the output is the complex voltages of both polarisations
// and/or Stokes I or IQUV, summed over n_int channel samples; incoherent beams form Stokes
// parameters per station and sum them.  The beam phase is formed like the fine delay: the
// angle f_c * dtau in double precision, reduced, then rotated in single precision.
//
// Coherent beams as a matrix product per channel and polarisation p:
//     beam[b][t] = sum_s w[b][s] Z[s*P + p][t]
// with K = the stations' interleaved (re, im) values:
//     Re = A_re . B,  A_re[b] = (Re w_s, -Im w_s)_s
//     Im = A_im . B,  A_im[b] = (Im w_s,  Re w_s)_s,   B[t] = (Re Z_s(t), Im Z_s(t))_s
// on v_mfma_f32_32x32x16_f16 tiles (32 beams x 32 samples), both the weights and the data
// split into fp16 hi + lo (products hh + hl + lh, FP32 accumulation; the dropped lo*lo term
// is below 2^-22 relative).  Time is the output (N) dimension, so each 32-sample block of a
// channel is an independent product: the block is staged in LDS with stations contiguous per
// sample, each wave owns one 32-beam tile with its weight fragments in registers, and the
// epilogue forms voltages / Stokes / sums over time directly from the accumulators.  The same
// LDS block gives the incoherent Stokes sums.
#include "cobalt_internal.h"

namespace cobalt {
namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef unsigned uintx4 __attribute__((ext_vector_type(4)));

constexpr int kBT = 32;                 // samples per block (one K block of the layout)

// hi = fp16(v), lo = fp16(v - hi) for a pair
__device__ __forceinline__ void split_h2(float a, float b, unsigned& hi, unsigned& lo) {
    const _Float16 ha = (_Float16)a, hb = (_Float16)b;
    const half2v h = {ha, hb};
    const half2v l = {(_Float16)(a - (float)ha), (_Float16)(b - (float)hb)};
    hi = __builtin_bit_cast(unsigned, h);
    lo = __builtin_bit_cast(unsigned, l);
}

// LDS words per (plane, pol, sample) row: stations padded to 8k, plus 4 words so that rows of
// consecutive samples start in different 16-byte bank groups
template <int KS>
constexpr int row_words() { return 8 * KS + 4; }

template <int KS>
__global__ __launch_bounds__(256, 1) void beam_kernel(BeamArgs a) {
    constexpr int RW = row_words<KS>();
    constexpr int kBuf = 2 * 2 * kBT * RW;              // words per staged block: [plane][pol][t][RW]
    __shared__ __attribute__((aligned(16))) unsigned sm[2 * kBuf];   // double buffer
    __shared__ float inc_part[8][4][kBT];               // incoherent partial sums [s-group][stokes][t]

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t ch = blockIdx.x;                      // sb * C + c
    const int sb = (int)(ch / a.C), c = (int)(ch % a.C);
    const int bt = blockIdx.y * 4 + wv;                 // beam tile of this wave
    const bool do_inc = a.incoherent != nullptr && blockIdx.y == 0;
    const char* chan = (const char*)a.chan + ch * a.chan_stride;

    // ---- weights of this wave's beams: fp16 hi/lo fragments for every k-step ----
    const double f_c = a.f_sb[sb] + (double)(c - a.C / 2) * a.df;
    uintx4 are_h[KS], are_l[KS], aim_h[KS], aim_l[KS];
    {
        const int b = bt * 32 + (lane & 31);
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int s = 8 * ks + 4 * (lane >> 5) + u;
                float wr = 0.f, wi = 0.f;
                if (b < a.NB && s < a.S) {
                    const double cyc = f_c * a.dtau[(int64_t)b * a.S + s];
                    const float r = (float)(cyc - rint(cyc));
                    wr = __builtin_amdgcn_cosf(r);
                    wi = __builtin_amdgcn_sinf(r);
                }
                unsigned h0, l0, h1, l1;
                split_h2(wr, -wi, h0, l0);
                split_h2(wi, wr, h1, l1);
                are_h[ks][u] = h0;
                are_l[ks][u] = l0;
                aim_h[ks][u] = h1;
                aim_l[ks][u] = l1;
            }
        }
    }

    // ---- staging: piece pc = (plane, row, 4-sample group) of 16 bytes; a block's pieces are
    // loaded into registers before the previous block's products and written to LDS after
    // them, so the loads overlap the MFMAs ----
    const int M = a.S * 2;
    const int n_pieces = 2 * M * (kBT / 4);             // <= 256 KS, i.e. KS per thread
    constexpr int kPieces = (2 * 2 * 8 * KS * (kBT / 4) + 255) / 256;
    uint4 pre[kPieces];
    auto load = [&](int kb) {
        const char* blk = chan + (int64_t)kb * (2 * M * 128);
#pragma unroll
        for (int i = 0; i < kPieces; ++i) {
            const int pc = tid + 256 * i;
            if (pc < n_pieces) {
                const int pl = pc / (M * 8), rem = pc % (M * 8);
                pre[i] = *(const uint4*)(blk + (int64_t)pl * (M * 128) + (rem >> 3) * 128 + (rem & 7) * 16);
            }
        }
    };
    auto store = [&](unsigned* buf) {
#pragma unroll
        for (int i = 0; i < kPieces; ++i) {
            const int pc = tid + 256 * i;
            if (pc < n_pieces) {
                const int pl = pc / (M * 8), rem = pc % (M * 8), row = rem >> 3, g = rem & 7;
                unsigned* dst = buf + ((pl * 2 + (row & 1)) * kBT + 4 * g) * RW + (row >> 1);
                dst[0] = pre[i].x;
                dst[RW] = pre[i].y;
                dst[2 * RW] = pre[i].z;
                dst[3 * RW] = pre[i].w;
            }
        }
    };
    // zero the station padding once in both buffers
    for (int i = tid; i < 2 * 2 * 2 * kBT; i += 256) {
        unsigned* r = sm + (i / (2 * 2 * kBT)) * kBuf + (i % (2 * 2 * kBT)) * RW;
        for (int s = a.S; s < 8 * KS; ++s) r[s] = 0u;
    }
    const int n_kb = a.n_kb;
    const float vscale = a.vscale;
    const int nS = a.n_stokes;
    const int n_out = a.n_c / a.n_int;

    __syncthreads();
    if (n_kb > 0) {
        load(0);
        store(sm);
    }
    for (int kb = 0; kb < n_kb; ++kb) {
        unsigned* buf = sm + (kb & 1) * kBuf;
        __syncthreads();                                // block kb is in LDS; buffer kb+1 is free
        if (kb + 1 < n_kb) load(kb + 1);
        const int t_lane = lane & 31, tb = kb * kBT;

        // ---- coherent: 32 beams x 32 samples, both polarisations ----
        if (bt * 32 < a.NB) {
            floatx16 re[2], im[2];
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                re[p] = floatx16{};
                im[p] = floatx16{};
            }
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                half8 Bh[2], Bl[2];
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    const int off = (p * kBT + t_lane) * RW + 8 * ks + 4 * (lane >> 5);
                    Bh[p] = __builtin_bit_cast(half8, *(const uintx4*)(buf + off));                 // plane 0 (hi)
                    Bl[p] = __builtin_bit_cast(half8, *(const uintx4*)(buf + 2 * kBT * RW + off));  // plane 1 (lo)
                }
                const half8 Ah_re = __builtin_bit_cast(half8, are_h[ks]), Ah_im = __builtin_bit_cast(half8, aim_h[ks]);
                const half8 Al_re = __builtin_bit_cast(half8, are_l[ks]), Al_im = __builtin_bit_cast(half8, aim_l[ks]);
                // four independent accumulators between dependent products
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    re[p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ah_re, Bh[p], re[p], 0, 0, 0);
                    im[p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ah_im, Bh[p], im[p], 0, 0, 0);
                }
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    re[p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ah_re, Bl[p], re[p], 0, 0, 0);
                    im[p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Ah_im, Bl[p], im[p], 0, 0, 0);
                }
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    re[p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Al_re, Bh[p], re[p], 0, 0, 0);
                    im[p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Al_im, Bh[p], im[p], 0, 0, 0);
                }
            }
            const int t = tb + t_lane;
            const bool tvalid = t < a.n_c;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int b = bt * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const bool bvalid = b < a.NB;
                const float xr = re[0][r] * vscale, xi = im[0][r] * vscale;
                const float yr = re[1][r] * vscale, yi = im[1][r] * vscale;
                if (a.voltages && bvalid && tvalid) {
                    float2* vo = (float2*)a.voltages + ((ch * a.NB + b) * 2) * (int64_t)a.n_c;
                    vo[t] = make_float2(xr, xi);
                    vo[a.n_c + t] = make_float2(yr, yi);
                }
                if (a.coherent) {
                    // Stokes of this (beam, sample); samples past N_c contribute zero
                    const float xx = xr * xr + xi * xi, yy = yr * yr + yi * yi;
                    float st4[4] = {xx + yy, xx - yy, 2.f * (xr * yr + xi * yi), 2.f * (xi * yr - xr * yi)};
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        if (k >= nS) break;
                        float v = tvalid ? st4[k] : 0.f;
                        const int ni = a.n_int < kBT ? a.n_int : kBT;
                        for (int m = 1; m < ni; m <<= 1) v += __shfl_xor(v, m, 64);    // within 32-lane halves
                        if (bvalid && (t_lane % ni) == 0 && tvalid) {
                            float* so = (float*)a.coherent + ((ch * a.NB + b) * nS + k) * (int64_t)n_out;
                            const int to = t / a.n_int;
                            if (a.n_int <= kBT || (t % a.n_int) == 0) so[to] = v;
                            else so[to] += v;                   // same workgroup, blocks in order
                        }
                    }
                }
            }
        }

        // ---- incoherent: sum over stations of per-station Stokes (one workgroup per channel) ----
        if (do_inc) {
            const int t = tid & 31, grp = tid >> 5;         // 8 groups of stations
            float acc[4] = {0.f, 0.f, 0.f, 0.f};
            for (int s = grp; s < a.S; s += 8) {
                float x[2], y[2];
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    const unsigned hw = buf[(p * kBT + t) * RW + s], lw = buf[(2 * kBT + p * kBT + t) * RW + s];
                    const half2v h = __builtin_bit_cast(half2v, hw), l = __builtin_bit_cast(half2v, lw);
                    const float vr = ((float)h.x + (float)l.x) * vscale, vi = ((float)h.y + (float)l.y) * vscale;
                    if (p == 0) { x[0] = vr; x[1] = vi; } else { y[0] = vr; y[1] = vi; }
                }
                const float xx = x[0] * x[0] + x[1] * x[1], yy = y[0] * y[0] + y[1] * y[1];
                acc[0] += xx + yy;
                acc[1] += xx - yy;
                acc[2] += 2.f * (x[0] * y[0] + x[1] * y[1]);
                acc[3] += 2.f * (x[1] * y[0] - x[0] * y[1]);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) inc_part[grp][k][t] = acc[k];
            __syncthreads();
            if (tid < 32 * nS) {
                const int k = tid >> 5, tt = tid & 31;
                float v = 0.f;
#pragma unroll
                for (int g2 = 0; g2 < 8; ++g2) v += inc_part[g2][k][tt];
                const int tg = tb + tt;
                if (tg >= a.n_c) v = 0.f;
                const int ni = a.n_int < kBT ? a.n_int : kBT;
                for (int m = 1; m < ni; m <<= 1) v += __shfl_xor(v, m, 64);
                if ((tt % ni) == 0 && tg < a.n_c) {
                    float* so = (float*)a.incoherent + (ch * nS + k) * (int64_t)n_out;
                    const int to = tg / a.n_int;
                    if (a.n_int <= kBT || (tg % a.n_int) == 0) so[to] = v;
                    else so[to] += v;
                }
            }
            __syncthreads();                                // inc_part reused next block
        }
        if (kb + 1 < n_kb) store(sm + ((kb + 1) & 1) * kBuf);
    }
}

template <int KS>
hipError_t launch_ks(const BeamArgs& a, hipStream_t st) {
    const dim3 grid((unsigned)a.n_chan, (unsigned)((a.NB + 127) / 128)), block(256);
    hipLaunchKernelGGL((beam_kernel<KS>), grid, block, 0, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_beamformer(const BeamArgs& a, hipStream_t st) {
    if (a.n_chan == 0) return hipSuccess;
    switch ((a.S + 7) / 8) {
        case 1: return launch_ks<1>(a, st);
        case 2: return launch_ks<2>(a, st);
        case 3: return launch_ks<3>(a, st);
        case 4: return launch_ks<4>(a, st);
        case 5: return launch_ks<5>(a, st);
        case 6: return launch_ks<6>(a, st);
        case 7: return launch_ks<7>(a, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace cobalt

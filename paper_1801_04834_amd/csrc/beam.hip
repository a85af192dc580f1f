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

// (a, b) -> (-b, a) on packed fp16 pairs: (Re w, -Im w) -> (Im w, Re w).  One packed max of a
// register with itself, the low result taking the negated high half and the high result the low
// half: exact for both the hi and the lo part of the split (fp16 denormals are kept).
__device__ __forceinline__ uintx4 re_to_im(uintx4 d) {
    uintx4 r;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        asm("v_pk_max_f16 %0, %1, %1 op_sel:[1,1] op_sel_hi:[0,0] neg_lo:[1,1]" : "=v"(r[e]) : "v"(d[e]));
    return r;
}

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Waves per SIMD the register budget is set for: three workgroups per CU where the LDS (two
// staged blocks of 16 KS rows) and the registers of up to 48 stations allow it.
template <int KS>
constexpr int beam_waves() { return KS <= 6 ? 3 : 2; }

template <int KS, int NS, bool VOLT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(beam_waves<KS>()))) void beam_kernel(BeamArgs a) {
    // one staged block = the channelised K block with its rows regrouped by polarisation:
    // [plane][pol][station][32 samples] words, 8 KS station rows per polarisation (padding rows
    // stay zero), so that consecutive stations of one polarisation are consecutive rows
    constexpr int kS8 = 8 * KS;                         // station rows per polarisation
    constexpr int kRows = 2 * kS8;
    constexpr int kPlaneW = kRows * kBT;
    constexpr int kBuf = 2 * kPlaneW;
    __shared__ __attribute__((aligned(1024))) unsigned sm[2 * kBuf];   // double buffer

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t ch = blockIdx.x;                      // sb * C + c
    const int sb = (int)(ch / a.C), c = (int)(ch % a.C);
    const int bt = blockIdx.y * 4 + wv;                 // beam tile of this wave
    const bool do_inc = a.incoherent != nullptr && blockIdx.y == 0;
    const char* chan = (const char*)a.chan + ch * a.chan_stride;

    // ---- weights of this wave's beams: fp16 hi/lo fragments for every k-step ----
    const double f_c = a.f_sb[sb] + (double)(c - a.C / 2) * a.df;
    // only the Re-part fragments are kept: the Im part (Im w, Re w) is (Re w, -Im w) with the
    // halves swapped and the new low half negated, rebuilt per k-step in registers
    uintx4 are_h[KS], are_l[KS];
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
                unsigned h0, l0;
                split_h2(wr, -wi, h0, l0);
                are_h[ks][u] = h0;
                are_l[ks][u] = l0;
            }
        }
    }

    // ---- staging: the block's rows go global -> LDS directly (global_load_lds, 16 bytes per
    // lane, one instruction = 8 LDS rows, each lane's source row chosen so that LDS row
    // p kS8 + s holds global row 2 s + p); the next block is requested before this block's
    // products.  Fragments are then gathered per station row (4-byte reads, paired). ----
    const int M = a.S * 2;
    constexpr int n_inst = kRows / 8;                   // per plane
    // Eight LDS rows of one instruction are 8 consecutive stations of one polarisation (8 divides
    // kS8), i.e. global rows 2 (st0 + l) + pol, l = lane / 8: the lane's part of the source
    // offset is the same for every instruction and the rest is wave-uniform.
    const int wvu = __builtin_amdgcn_readfirstlane(wv);
    const int lst = lane >> 3;
    const unsigned lane_off = (unsigned)(lst * 256 + (lane & 7) * 16);
    constexpr int kIt = (2 * n_inst + 3) / 4;           // instructions per wave and block
    int src_off[kIt], dst_off[kIt];                     // wave-uniform, fixed for the kernel
    bool live[kIt];
#pragma unroll
    for (int it = 0; it < kIt; ++it) {
        const int i = wvu + 4 * it;
        const int pl = i / n_inst, j = i % n_inst;
        const int pol = (8 * j) / kS8, st0 = (8 * j) % kS8;
        src_off[it] = (pl * M + 2 * st0 + pol) * 128;
        dst_off[it] = pl * kPlaneW + j * 256;
        live[it] = i < 2 * n_inst && st0 + lst < a.S;
    }
    auto issue = [&](int kb, unsigned* buf) {
        const char* blk = chan + (int64_t)kb * (2 * M * 128);
#pragma unroll
        for (int it = 0; it < kIt; ++it)
            if (live[it])
                __builtin_amdgcn_global_load_lds((const void*)(blk + src_off[it] + lane_off),
                                                 (lds_ptr_t)(buf + dst_off[it]), 16, 0, 0);
    };
    // zero the padding rows (stations S .. kS8 - 1 of each polarisation) of both planes of both
    // buffers once
    const int npad = kS8 - a.S;
    for (int i = tid; i < 2 * 2 * 2 * npad * kBT; i += 256) {
        const int w = i % kBT, r = (i / kBT) % npad, pol = (i / (kBT * npad)) % 2, pl = (i / (kBT * npad * 2)) % 2,
                  bufi = i / (kBT * npad * 4);
        sm[bufi * kBuf + pl * kPlaneW + (pol * kS8 + a.S + r) * kBT + w] = 0u;
    }
    const int n_kb = a.n_kb;
    const float vscale = a.vscale;
    constexpr int nS = NS;                              // Stokes parameters: 1 (I) or 4 (IQUV)
    const float sscale = vscale * vscale;               // Stokes are quadratic in the voltages
    const int n_out = a.n_c / a.n_int;
    const int g = a.n_int < kBT ? a.n_int : kBT;        // samples summed inside one block
    const int gsh = __builtin_ctz((unsigned)g);         // g is a power of two
    // output index of a window starting at sample t: t / n_int (a shift for n_int <= 32)
    auto out_index = [&](int t) { return a.n_int <= kBT ? (t >> gsh) : t / a.n_int; };
    // per-channel output bases (32-bit offsets below)
    float* const co_ch = a.coherent ? (float*)a.coherent + ch * (int64_t)n_out * nS * a.NB : nullptr;
    float2* const vo_ch = a.voltages ? (float2*)a.voltages + ch * (int64_t)a.n_c * 2 * a.vstride : nullptr;
    float* const io_ch = a.incoherent ? (float*)a.incoherent + ch * (int64_t)n_out * nS : nullptr;
    const int hb = lane >> 5;
    const int b = bt * 32 + (lane & 31);                // this lane's beam (output column)
    const bool bvalid = b < a.NB;

    // Stokes of one (beam, sample) from the two polarisations' voltages (unscaled)
    auto stokes = [&](float xr, float xi, float yr, float yi, float* st) {
        const float xx = xr * xr + xi * xi, yy = yr * yr + yi * yi;
        st[0] = xx + yy;
        if constexpr (NS == 4) {
            st[1] = xx - yy;
            st[2] = 2.f * (xr * yr + xi * yi);
            st[3] = 2.f * (xi * yr - xr * yi);
        }
    };
    // v of lane i plus v of lane i ^ 32
    auto add_halves = [&](float v) {
        const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
        return __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
    };
    // write or accumulate (windows longer than a block: blocks of one workgroup run in order)
    auto put = [&](float* o, int tstart, float v) {
        if (a.n_int <= kBT || tstart % a.n_int == 0) *o = v;
        else *o += v;
    };
    // incoherent partial sums of a block, [buffer][wave][sample][stokes]: wave w holds the sums
    // over the stations of groups 2w and 2w + 1 (station s is in group s % 8)
    __shared__ float inc_p[2][4][kBT][NS];
    // after a barrier: the four partial sums of each sample of block kbp in a fixed order, then
    // the sums over windows of g samples (32 lanes per Stokes parameter, from wave 0 on)
    auto inc_finish = [&](int kbp) {
        const int idx = wv * 64 + lane, k = idx / kBT, tl = idx % kBT;
        if (k >= NS) return;
        const int t = kbp * kBT + tl;
        const int bi = kbp & 1;
        float x = t < a.n_c ? ((inc_p[bi][0][tl][k] + inc_p[bi][1][tl][k]) + (inc_p[bi][2][tl][k] + inc_p[bi][3][tl][k])) * sscale : 0.f;
        for (int m = 1; m < g; m <<= 1) x += __shfl_xor(x, m, 64);
        if ((tl & (g - 1)) == 0 && t < a.n_c) put(io_ch + out_index(t) * nS + k, t, x);
    };

    __syncthreads();
    if (n_kb > 0) issue(0, sm);
    for (int kb = 0; kb < n_kb; ++kb) {
        unsigned* buf = sm + (kb & 1) * kBuf;
        __builtin_amdgcn_s_waitcnt(0);                  // this wave's transfers of block kb have landed
        __syncthreads();                                // ... and everyone's; buffer kb+1 is free
        if (do_inc && kb > 0) inc_finish(kb - 1);
        if (kb + 1 < n_kb) issue(kb + 1, sm + ((kb + 1) & 1) * kBuf);
        const int tb = kb * kBT;

        // ---- coherent: D[t][b] = data (32 samples x K) . weights (K x 32 beams) ----
        if ((VOLT || a.coherent) && bt * 32 < a.NB) {
            floatx16 re[2], im[2];
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                re[p] = floatx16{};
                im[p] = floatx16{};
            }
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                half8 Dh[2], Dl[2];
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    // stations 8 ks + 4 hb + u (u = 0..3), sample lane % 32: LDS rows p kS8 + s,
                    // read in pairs straight into the fragment's adjacent registers
                    uintx4 h, l;
                    const int w0 = (p * kS8 + 8 * ks + 4 * hb) * kBT + (lane & 31);
#pragma unroll
                    for (int u = 0; u < 4; ++u) h[u] = buf[w0 + u * kBT];
#pragma unroll
                    for (int u = 0; u < 4; ++u) l[u] = buf[kPlaneW + w0 + u * kBT];
                    Dh[p] = __builtin_bit_cast(half8, h);
                    Dl[p] = __builtin_bit_cast(half8, l);
                }
                const half8 Wh_re = __builtin_bit_cast(half8, are_h[ks]), Wh_im = __builtin_bit_cast(half8, re_to_im(are_h[ks]));
                const half8 Wl_re = __builtin_bit_cast(half8, are_l[ks]), Wl_im = __builtin_bit_cast(half8, re_to_im(are_l[ks]));
                // four independent accumulators between dependent products
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    re[p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Dh[p], Wh_re, re[p], 0, 0, 0);
                    im[p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Dh[p], Wh_im, im[p], 0, 0, 0);
                }
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    re[p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Dl[p], Wh_re, re[p], 0, 0, 0);
                    im[p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Dl[p], Wh_im, im[p], 0, 0, 0);
                }
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    re[p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Dh[p], Wl_re, re[p], 0, 0, 0);
                    im[p] = __builtin_amdgcn_mfma_f32_32x32x16_f16(Dh[p], Wl_im, im[p], 0, 0, 0);
                }
            }
            // register r of lane i holds sample t = 8 (r/4) + 4 (i/32) + r%4 of beam b
            // padding beams of a row (NB <= b < vstride) that this tile covers get zeros, so a
            // row padded to whole 128-byte lines is written as whole lines
            if (VOLT && b < a.vstride) {
                const float vs = bvalid ? vscale : 0.f;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int t = tb + 8 * (r >> 2) + 4 * hb + (r & 3);
                    if (t < a.n_c) {
                        const unsigned o = (unsigned)(t * 2 * a.vstride + b);
                        const float x0 = bvalid ? re[0][r] : 0.f, y0 = bvalid ? im[0][r] : 0.f;
                        const float x1 = bvalid ? re[1][r] : 0.f, y1 = bvalid ? im[1][r] : 0.f;
                        vo_ch[o] = make_float2(x0 * vs, y0 * vs);
                        vo_ch[o + a.vstride] = make_float2(x1 * vs, y1 * vs);
                    }
                }
            }
            if (a.coherent) {
                // Stokes per register group q (samples 8q + 4 hb + u, u = 0..3), summed over g
                // consecutive samples: runs of up to 4 sit in one lane's group; runs of 8 span
                // the two lane halves; longer runs also span groups.  All register indices are
                // compile-time; g and nS only select.
                const int per = g >= 8 ? g / 8 : 1;
                const bool full = tb + kBT <= a.n_c;            // no sample past N_c (uniform)
                float part[NS] = {};
                // Stokes I over windows of 8 or more samples in a whole block: the squares go
                // straight into the window sum, four FMAs per sample, nothing to mask
                const bool fast = NS == 1 && g >= 8 && full;
#pragma unroll
                for (int q = 0; q < 4 && fast; ++q) {
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int r = 4 * q + u;
                        part[0] = fmaf(re[0][r], re[0][r], part[0]);
                        part[0] = fmaf(im[0][r], im[0][r], part[0]);
                        part[0] = fmaf(re[1][r], re[1][r], part[0]);
                        part[0] = fmaf(im[1][r], im[1][r], part[0]);
                    }
                    if ((q + 1) % per == 0) {
                        const int t = tb + 8 * (q + 1 - per);
                        const float v = add_halves(part[0]) * sscale;
                        if (hb == 0 && bvalid) put(co_ch + (unsigned)(out_index(t) * a.NB + b), t, v);
                        part[0] = 0.f;
                    }
                }
#pragma unroll
                for (int q = 0; q < 4 && !fast; ++q) {
                    float st[4][NS];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int r = 4 * q + u;
                        stokes(re[0][r], im[0][r], re[1][r], im[1][r], st[u]);
                        if (!full && tb + 8 * q + 4 * hb + u >= a.n_c)
#pragma unroll
                            for (int k = 0; k < NS; ++k) st[u][k] = 0.f;
                    }
                    if (g <= 4) {
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int t = tb + 8 * q + 4 * hb + u;
                            const bool lead = (u & (g - 1)) == 0;
#pragma unroll
                            for (int k = 0; k < NS; ++k) {
                                float v = st[u][k];
#pragma unroll
                                for (int w = 1; w < 4; ++w)
                                    if (u + w < 4 && w < g) v += st[u + w][k];
                                if (lead && bvalid && t < a.n_c)
                                    co_ch[(unsigned)((out_index(t) * nS + k) * a.NB + b)] = v * sscale;
                            }
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < NS; ++k)
                            part[k] += st[0][k] + st[1][k] + st[2][k] + st[3][k];
                        if ((q + 1) % per == 0) {              // window of g samples complete
                            const int t = tb + 8 * (q + 1 - per);
#pragma unroll
                            for (int k = 0; k < NS; ++k) {
                                const float v = add_halves(part[k]) * sscale;
                                if (hb == 0 && bvalid && t < a.n_c)
                                    put(co_ch + (unsigned)((out_index(t) * nS + k) * a.NB + b), t, v);
                            }
#pragma unroll
                            for (int k = 0; k < NS; ++k) part[k] = 0.f;
                        }
                    }
                }
            }
        }

        // ---- incoherent: lane (half hb, sample tl) of wave w sums stations 8 ks + 2 w + hb; one
        // read of a wave covers two station rows of 32 samples.  For Stokes I every read is at a
        // fixed offset from one lane base (the hi and lo words of a station row in one paired
        // read), the padding rows (stations S .. 8 KS - 1) being zero and adding nothing ----
        if (do_inc) {
            const int tl = lane & 31, grp = 2 * wv + hb;
            const unsigned* q = buf + grp * kBT + tl;
            float acc[NS] = {};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int s = grp + 8 * ks;
                if (NS != 1 && s >= a.S) continue;
                float v[2][2];
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    unsigned hw, lw;
                    if constexpr (NS == 1) {
                        hw = q[(p * kS8 + 8 * ks) * kBT];
                        lw = q[kPlaneW + (p * kS8 + 8 * ks) * kBT];
                    } else {
                        hw = buf[(p * kS8 + s) * kBT + tl];
                        lw = buf[kPlaneW + (p * kS8 + s) * kBT + tl];
                    }
                    // hi + lo of the (re, im) halves in one mixed-precision FMA each (exact in FP32)
                    asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,1]" : "=v"(v[p][0]) : "v"(hw), "v"(lw));
                    asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,1] op_sel_hi:[1,0,1]" : "=v"(v[p][1]) : "v"(hw), "v"(lw));
                }
                if constexpr (NS == 1) {
                    acc[0] = fmaf(v[0][0], v[0][0], acc[0]);
                    acc[0] = fmaf(v[0][1], v[0][1], acc[0]);
                    acc[0] = fmaf(v[1][0], v[1][0], acc[0]);
                    acc[0] = fmaf(v[1][1], v[1][1], acc[0]);
                } else {
                    float st4[NS];
                    stokes(v[0][0], v[0][1], v[1][0], v[1][1], st4);
#pragma unroll
                    for (int k = 0; k < NS; ++k) acc[k] += st4[k];
                }
            }
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                const float x = add_halves(acc[k]);
                if (hb == 0) inc_p[kb & 1][wv][tl][k] = x;
            }
        }
    }
    if (do_inc && n_kb > 0) {
        __syncthreads();
        inc_finish(n_kb - 1);
    }
}

// VOLT: the voltage output is compiled in only where voltages are asked for
template <int KS>
hipError_t launch_ks(const BeamArgs& a, hipStream_t st) {
    const dim3 grid((unsigned)a.n_chan, (unsigned)((a.NB + 127) / 128)), block(256);
    const bool v = a.voltages != nullptr;
    if (a.n_stokes == 1) {
        if (v) hipLaunchKernelGGL((beam_kernel<KS, 1, true>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((beam_kernel<KS, 1, false>), grid, block, 0, st, a);
    } else {
        if (v) hipLaunchKernelGGL((beam_kernel<KS, 4, true>), grid, block, 0, st, a);
        else hipLaunchKernelGGL((beam_kernel<KS, 4, false>), grid, block, 0, st, a);
    }
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

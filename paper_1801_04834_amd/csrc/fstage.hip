// F stage of the FX correlator for gfx950: unpack -> polyphase FIR (history carried) ->
// 64-point FFT -> fine delay compensation + bandpass correction -> transpose to the
// cross-station layout with precision conversion.
//
// The paper's correlator pipeline channelises each subband with FIR filters feeding an
// FFT, carries the FIR history into the next block, applies fine delay compensation and
// bandpass correction, and transposes on write-back so the correlator can work across
// antenna fields ("Signal processing with GPU kernels", sec. 7.5).  Samples arrive as
// fixed point and are converted to float ("Processing steps", sec. 3.2).  The delay phase
// is formed in double precision; the rotation runs in single precision (sec. 7.5, sec. 8).
//
// Work decomposition (one wave64 per workgroup):
//   workgroup = one input stream (station, polarisation, subband) x one chunk of 256
//   channel samples, processed in passes of 32 channel samples.
//   FIR:   lane p is FIR phase p; it keeps a 15-row sliding window in registers, so every
//          input sample is read from HBM once (coalesced 64-lane rows).
//   FFT:   the first radix-2 decimation-in-frequency stage runs across lanes p and p+32
//          with v_permlane32_swap (two channel samples per swap); the two 32-point halves
//          go through LDS so that lane (j, h) owns one 32-point DFT in registers.
//   Delay: per (channel, sample) the phase in cycles f_c * tau(j) is formed with one FP64
//          FMA and reduced with FP64 rint; the reduced phase is rotated in FP32 with the
//          hardware sin/cos (argument in revolutions).
//   Store: lanes with equal h write 32 consecutive channel samples of one channel row.
#include "cobalt_internal.h"

namespace cobalt {
namespace {

constexpr int kPass = 32;                 // channel samples per pass (= one K block)
static_assert(kPass == kKBlock, "a pass writes exactly one K block per channel");
constexpr int kChunk = kFChunk;           // channel samples per workgroup (8 passes)
constexpr int kRowF2 = 68;                // complex staging row (float2): two 32-point halves, 16 B apart
constexpr int kHalfF2 = 34;
constexpr int kRowF1 = 72;                // split staging row (floats): conflict-free 16-byte column reads
constexpr int kHalfF1 = 36;

constexpr double kPi = 3.141592653589793238462643383279502884;

constexpr double taylor_sin(double x) {
    double term = x, sum = x;
    for (int n = 1; n < 24; ++n) { term *= -x * x / ((2.0 * n) * (2.0 * n + 1.0)); sum += term; }
    return sum;
}
constexpr double taylor_cos(double x) {
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 24; ++n) { term *= -x * x / ((2.0 * n - 1.0) * (2.0 * n)); sum += term; }
    return sum;
}
// cos and sin of 2*pi*t/64 rounded to float, t in [0, 64)
constexpr float tw_cos(int t) {
    const int q = t / 16, r = t % 16;
    const double th = 2.0 * kPi * r / 64.0, c = taylor_cos(th), s = taylor_sin(th);
    return (float)(q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s);
}
constexpr float tw_sin(int t) {
    const int q = t / 16, r = t % 16;
    const double th = 2.0 * kPi * r / 64.0, c = taylor_cos(th), s = taylor_sin(th);
    return (float)(q == 0 ? s : q == 1 ? c : q == 2 ? -s : -c);
}

// (re + i im) * exp(-2 pi i t / 64), t a compile-time constant
template <int t>
__device__ __forceinline__ void rot_w64(float& re, float& im) {
    if constexpr (t == 0) {
        return;
    } else if constexpr (t == 16) {
        const float r = re;
        re = im;
        im = -r;
    } else if constexpr (t == 8) {
        constexpr float c = tw_cos(8);
        const float r = re;
        re = (r + im) * c;
        im = (im - r) * c;
    } else if constexpr (t == 24) {
        constexpr float c = tw_sin(24);   // = 1/sqrt(2); cos(3 pi/4) = -c
        const float r = re;
        re = (im - r) * c;
        im = -(im + r) * c;
    } else {
        constexpr float c = tw_cos(t), s = tw_sin(t);
        const float r = re;
        re = r * c + im * s;
        im = im * c - r * s;
    }
}

// One radix-2 decimation-in-frequency stage of a 32-point DFT (butterfly span `span`).
template <int span, int k>
__device__ __forceinline__ void dif_group(float (&re)[32], float (&im)[32], int start) {
    if constexpr (k < span) {
        const int i0 = start + k, i1 = i0 + span;
        const float ar = re[i0], ai = im[i0], br = re[i1], bi = im[i1];
        re[i0] = ar + br;
        im[i0] = ai + bi;
        float dr = ar - br, di = ai - bi;
        rot_w64<k * (32 / span)>(dr, di);
        re[i1] = dr;
        im[i1] = di;
        dif_group<span, k + 1>(re, im, start);
    }
}
template <int span>
__device__ __forceinline__ void dif_stage(float (&re)[32], float (&im)[32]) {
#pragma unroll
    for (int start = 0; start < 32; start += 2 * span) dif_group<span, 0>(re, im, start);
}
// Forward 32-point DFT, natural-order input; output element i holds bin bitrev5(i).
__device__ __forceinline__ void fft32(float (&re)[32], float (&im)[32]) {
    dif_stage<16>(re, im);
    dif_stage<8>(re, im);
    dif_stage<4>(re, im);
    dif_stage<2>(re, im);
    dif_stage<1>(re, im);
}
constexpr int bitrev5(int i) {
    return ((i & 1) << 4) | ((i & 2) << 2) | (i & 4) | ((i & 8) >> 2) | ((i & 16) >> 4);
}

template <int ST> struct Samp;
template <> struct Samp<ST_CI16> {
    using raw_t = uint32_t;
    static __device__ __forceinline__ float2 cvt(raw_t w) {
        return make_float2((float)(int16_t)(w & 0xffffu), (float)((int32_t)w >> 16));
    }
};
template <> struct Samp<ST_CI8> {
    using raw_t = uint16_t;
    static __device__ __forceinline__ float2 cvt(raw_t w) {
        return make_float2((float)(int8_t)(w & 0xffu), (float)(int8_t)(w >> 8));
    }
};
template <> struct Samp<ST_CF32> {
    using raw_t = float2;
    static __device__ __forceinline__ float2 cvt(raw_t w) { return w; }
};

// One pass of input rows (32 rows x this lane's phase).  8-bit samples are packed two
// rows per VGPR (16-bit halves), wider samples take one element per row.
template <int ST, int C>
struct PassBuf {
    using raw_t = typename Samp<ST>::raw_t;
    raw_t v[kPass];
    // rows jb .. jb + 31 of this wave's phases: a wave-uniform base for the pass and per-lane
    // offsets lane + r*C, so the loads take a scalar base, one offset register and immediates
    __device__ __forceinline__ void load(const raw_t* __restrict__ in, int lane, int jb, int n_c) {
        const raw_t* __restrict__ rows = in + (int64_t)jb * C;
        if (jb + kPass <= n_c) {
#pragma unroll
            for (int r = 0; r < kPass; ++r) v[r] = rows[r * C + lane];
        } else {
#pragma unroll
            for (int r = 0; r < kPass; ++r) v[r] = jb + r < n_c ? rows[r * C + lane] : raw_t{};
        }
    }
    __device__ __forceinline__ raw_t get(int r) const { return v[r]; }
};
typedef unsigned short ushort2v __attribute__((ext_vector_type(2)));
template <int C>
struct PassBuf<ST_CI8, C> {
    ushort2v v[kPass / 2];
    __device__ __forceinline__ void load(const uint16_t* __restrict__ in, int lane, int jb, int n_c) {
        const uint16_t* __restrict__ rows = in + (int64_t)jb * C;
        if (jb + kPass <= n_c) {
#pragma unroll
            for (int r = 0; r < kPass; ++r) v[r / 2][r % 2] = rows[r * C + lane];
        } else {
#pragma unroll
            for (int r = 0; r < kPass; ++r) v[r / 2][r % 2] = jb + r < n_c ? rows[r * C + lane] : (uint16_t)0;
        }
    }
    __device__ __forceinline__ uint16_t get(int r) const { return v[r / 2][r % 2]; }
};

typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));

template <int OM> struct OutFmt;
template <> struct OutFmt<XM_FP32> { static constexpr int kPlanes = 1, kElem = 8; };
template <> struct OutFmt<XM_FP16_SPLIT> { static constexpr int kPlanes = 2, kElem = 4; };
template <> struct OutFmt<XM_INT8> { static constexpr int kPlanes = 1, kElem = 2; };

// exp(2 pi i r) for a phase r already reduced to [-1/2, 1/2] cycles (hardware sin/cos take
// the argument in revolutions)
__device__ __forceinline__ float2 phasor_rev(double cyc) {
    const float r = (float)(cyc - rint(cyc));
    return make_float2(__builtin_amdgcn_cosf(r), __builtin_amdgcn_sinf(r));
}

// Minimum waves per SIMD each instantiation is compiled for: 3 where the registers fit
// without spilling, 2 otherwise (the compiled register counts allow 3 everywhere at present;
// LDS then decides: 9 workgroups per CU for the complex FFT staging at 64 channels).
template <int ST, int OM, int C>
constexpr int fstage_waves() { return C == 64 && (ST == ST_CF32 || (ST == ST_CI16 && OM == XM_FP16_SPLIT)) ? 3 : 2; }

// C = 64: one wave per workgroup; lane p is FIR phase p and the 64-point FFT is the
// lane-pair stage + LDS + 32-point DFT per lane described above.
// C = 256: four waves per workgroup; wave m holds FIR phases 64m + p.  A radix-4
// decimation-in-frequency stage across the waves (through LDS) leaves wave r with
//   z_r[p] = exp(-2 pi i r p / 256) sum_m y[p + 64m] (-i)^(m r),
// whose 64-point DFT is bins k = 4k' + r of the 256-point DFT; that 64-point DFT then runs
// exactly as for C = 64.
template <int ST, int OM, int C>
__global__ __launch_bounds__(C) __attribute__((amdgpu_waves_per_eu(fstage_waves<ST, OM, C>()))) void fstage_kernel(FArgs a) {
    static_assert(C == 64 || C == 256, "64 or 256 channels");
    constexpr int kW = C / 64;                 // waves per workgroup
    constexpr int kHistC = kHistRows * C;      // history samples per stream
    using S_ = Samp<ST>;
    using raw_t = typename S_::raw_t;
    using O_ = OutFmt<OM>;
    // Per-wave FFT staging rows; for C = 256 the same memory first holds the radix-4
    // exchange (all waves' FIR outputs of half a pass).  8-bit input (VALU-bound) and 256
    // channels stage real and imaginary parts in turn through a float buffer, halving the LDS
    // per wave so that more waves fit a CU (measured 8.3 -> 7.9 ms per 8-bit block, 3.79 ->
    // 3.54 ms per 256-channel block); 16-bit and float input at 64 channels keep one complex
    // buffer (the split costs them ~2 %).
    constexpr bool kSplit = ST == ST_CI8 || C == 256;
    constexpr int kYl = kSplit ? kPass * kRowF1 : 2 * kPass * kRowF2;   // floats per wave
    // the radix-4 exchange of C = 256 goes in two halves of the pass's channel samples
    constexpr int kXj = kSplit ? kPass / 2 : kPass;
    constexpr int kXch = kW > 1 ? 2 * kW * kXj * 64 : 0;
    __shared__ __attribute__((aligned(16))) float lds_f[kW * kYl > kXch ? kW * kYl : kXch];
    // Bandpass x mode scale per channel, staged in LDS: reading it from global memory in the
    // store loop would put a vector-memory wait on every channel, and such a wait also waits
    // for the prefetched rows of the next pass.  (The first pass's barrier orders this write.)
    __shared__ float blds[C];

    const int lane = threadIdx.x & 63;
    const int wv = kW > 1 ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : 0;   // wave index
    float* const ylds = lds_f + wv * kYl;
    // grid order: input row fastest, so neighbouring rows of one channel K block are
    // written by concurrently running waves (contiguous in the K-blocked layout)
    const int row_in = (int)(blockIdx.x % (unsigned)a.M);               // input index s*P + p
    const int rest = (int)(blockIdx.x / (unsigned)a.M);
    const int chunk = rest % a.n_chunks;
    const int sb = rest / a.n_chunks;
    const int64_t st = (int64_t)row_in * a.SB + sb;                      // input stream (s*P + p)*SB + sb
    const int s = row_in >> 1;
    // wave-uniform bases; per-lane offsets below stay within 2^31 bytes
    // block window of this stream: its row, shifted by the station's coarse delay
    const raw_t* __restrict__ in = (const raw_t*)a.in + st * a.row_len + (a.coarse ? a.coarse[s] : 0);
    // flagged channel samples of this station and subband (one bit per channel sample)
    const uint32_t* __restrict__ cflag = a.cflag ? a.cflag + ((int64_t)s * a.SB + sb) * a.n_words : nullptr;
    const raw_t* __restrict__ hold = (const raw_t*)a.hist_old + st * kHistC;
    // this wave's FIR phases 64 wv .. 64 wv + 63
    const raw_t* __restrict__ inw = in + 64 * wv;
    const raw_t* __restrict__ holdw = hold + 64 * wv;
    // channelised layout [SB][C][n_kb][planes][M][32]: element (row, j) of channel c lives
    // in K block j/32 at position j%32 of the row
    char* __restrict__ out = (char*)a.out + ((int64_t)sb * C * a.n_kb * O_::kPlanes * a.M + row_in) * kKBlock * O_::kElem;
    const uint32_t cstride = (uint32_t)(a.n_kb * O_::kPlanes * a.M * kKBlock * O_::kElem);   // bytes between channels
    const uint32_t pstride = (uint32_t)(a.M * kKBlock * O_::kElem);                          // bytes between planes
    const uint32_t kbstride = (uint32_t)(O_::kPlanes * a.M * kKBlock * O_::kElem);           // bytes between K blocks
    const uint32_t ulane = (uint32_t)lane;

    // The last chunk of every stream writes the history for the next block: the final
    // (T-1)*C samples of [old history, block].
    if (chunk == a.n_chunks - 1) {
        raw_t* hnew = (raw_t*)a.hist_new + st * kHistC;
        for (int i = threadIdx.x; i < kHistC; i += C) {
            const int64_t t = a.N + i;
            hnew[i] = t < kHistC ? hold[t] : in[t - kHistC];
        }
    }

    for (int i = threadIdx.x; i < C; i += 64 * kW) blds[i] = a.bscale[i];
    float h[kT];
#pragma unroll
    for (int t = 0; t < kT; ++t) h[t] = a.fir[t * C + 64 * wv + lane];
    float rtw_c = 1.f, rtw_s = 0.f;            // radix-4 twiddle exp(-2 pi i wv lane / C) = (c, -s)
    if constexpr (kW > 1) sincospif(2.0f * (float)(wv * lane) / (float)C, &rtw_s, &rtw_c);

    float wsn, wcs;                            // exp(-2 pi i q / 64), q = lane mod 32
    sincospif((float)(lane & 31) / 32.0f, &wsn, &wcs);

    const double tau0 = a.delays[2 * s], tau1 = a.delays[2 * s + 1];
    const double fsb = a.f_sb[sb];
    const int jj = lane >> 1, hh = lane & 1;

    const int j0 = chunk * kChunk;
    const int jend = min(j0 + kChunk, a.pitch);

    raw_t tail[kHistRows];                     // raw samples of the 15 rows before the pass
    if (j0 >= kHistRows && j0 <= a.n_c) {
#pragma unroll
        for (int i = 0; i < kHistRows; ++i) tail[i] = inw[(uint32_t)((j0 - kHistRows + i) * C) + ulane];
    } else {
#pragma unroll
        for (int i = 0; i < kHistRows; ++i) {
            const int r = j0 - kHistRows + i;  // wave-uniform
            tail[i] = r < 0 ? holdw[(r + kHistRows) * C + lane] : r < a.n_c ? inw[r * C + lane] : raw_t{};
        }
    }

    // Rows of the next pass are requested right after the FIR has consumed the current ones,
    // so their HBM latency overlaps the FFT, delay and store work of this pass (8/16-bit
    // samples; float samples, 2 VGPRs each, are loaded at the top of the pass instead).
    constexpr bool kPrefetch = ST != ST_CF32;
    PassBuf<ST, C> nw;
    if constexpr (kPrefetch) nw.load(inw, lane, j0, a.n_c);

    for (int jb = j0; jb < jend; jb += kPass) {
        if constexpr (!kPrefetch) nw.load(inw, lane, jb, a.n_c);

        // ---- polyphase FIR: y_j[p] = sum_t h[t*C + p] x[(j - T + 1 + t)*C + p] ----
        // input-stationary: window row w feeds outputs j = w - t (taps in ascending t)
        float2 acc[kPass];
#pragma unroll
        for (int j = 0; j < kPass; ++j) acc[j] = make_float2(0.f, 0.f);
#pragma unroll
        for (int w = 0; w < kPass + kHistRows; ++w) {
            const float2 x = S_::cvt(w < kHistRows ? tail[w] : nw.get(w - kHistRows));
#pragma unroll
            for (int t = 0; t < kT; ++t) {
                const int j = w - t;
                if (j >= 0 && j < kPass) {
                    acc[j].x = fmaf(h[t], x.x, acc[j].x);
                    acc[j].y = fmaf(h[t], x.y, acc[j].y);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < kHistRows; ++i) tail[i] = nw.get(kPass - kHistRows + i);
        if constexpr (kPrefetch) {
            if (jb + kPass < jend) nw.load(inw, lane, jb + kPass, a.n_c);
        }

        // Channel samples past N_c and flagged ones (their FIR window reads a lost sample) are
        // written as zero: their FIR outputs are cleared here, so the FFT, rotation and
        // stores below carry zeros.  The mask is wave-uniform (bit jj = channel sample jb+jj).
        {
            uint32_t kill = cflag ? cflag[jb / kKBlock] : 0u;
            if (jb + kPass > a.n_c) kill |= ~((1u << (a.n_c - jb)) - 1u);   // 1 <= n_c - jb < 32 here
            if (kill) {
#pragma unroll
                for (int j = 0; j < kPass; ++j)
                    if ((kill >> j) & 1u) acc[j] = make_float2(0.f, 0.f);
            }
        }

        // ---- C = 256: radix-4 stage across the four waves (bins k = 4k' + wv remain) ----
        if constexpr (kW > 1) {
            float2* xch = (float2*)lds_f;                             // [wave m][j - j0][lane]
#pragma unroll
            for (int j0 = 0; j0 < kPass; j0 += kXj) {
#pragma unroll
                for (int j = j0; j < j0 + kXj; ++j) xch[(wv * kXj + j - j0) * 64 + lane] = acc[j];
                __syncthreads();
#pragma unroll
                for (int j = j0; j < j0 + kXj; ++j) {
                    const float2 a0 = xch[(0 * kXj + j - j0) * 64 + lane], a1 = xch[(1 * kXj + j - j0) * 64 + lane];
                    const float2 a2 = xch[(2 * kXj + j - j0) * 64 + lane], a3 = xch[(3 * kXj + j - j0) * 64 + lane];
                    float zr, zi;
                    if (wv == 0) {
                        zr = (a0.x + a2.x) + (a1.x + a3.x);
                        zi = (a0.y + a2.y) + (a1.y + a3.y);
                    } else if (wv == 2) {
                        zr = (a0.x + a2.x) - (a1.x + a3.x);
                        zi = (a0.y + a2.y) - (a1.y + a3.y);
                    } else {
                        // (a0 - a2) -+ i (a1 - a3) for wv = 1 / 3
                        const float ur = a0.x - a2.x, ui = a0.y - a2.y, vr = a1.x - a3.x, vi = a1.y - a3.y;
                        zr = wv == 1 ? ur + vi : ur - vi;
                        zi = wv == 1 ? ui - vr : ui + vr;
                    }
                    acc[j] = make_float2(zr * rtw_c + zi * rtw_s, zi * rtw_c - zr * rtw_s);
                }
                __syncthreads();                                      // the exchange is read before reuse
            }
        }

        // ---- first DIF stage across lanes p, p+32 (two channel samples per swap) ----
        // The stage's outputs go through LDS to the lanes that own the 32-point DFTs.
        float xr[32], xi[32];
        if constexpr (!kSplit) {
            float2* const yl = (float2*)ylds;
#pragma unroll
            for (int pr = 0; pr < kPass / 2; ++pr) {
                const float2 A = acc[2 * pr], B = acc[2 * pr + 1];
                const auto sr = __builtin_amdgcn_permlane32_swap(__float_as_uint(A.x), __float_as_uint(B.x), false, false);
                const auto si = __builtin_amdgcn_permlane32_swap(__float_as_uint(A.y), __float_as_uint(B.y), false, false);
                // lanes < 32: (y_j[q], y_j[q+32]) of j = 2pr; lanes >= 32: same for j = 2pr+1
                const float r0r = __uint_as_float(sr[0]), r1r = __uint_as_float(sr[1]);
                const float r0i = __uint_as_float(si[0]), r1i = __uint_as_float(si[1]);
                const float dr = r0r - r1r, di = r0i - r1i;
                const int row = 2 * pr + (lane >> 5), q = lane & 31;
                yl[row * kRowF2 + q] = make_float2(r0r + r1r, r0i + r1i);
                yl[row * kRowF2 + kHalfF2 + q] = make_float2(dr * wcs + di * wsn, di * wcs - dr * wsn);
            }
            __syncthreads();
            // ---- 32-point DFT of the even (h = 0) or odd (h = 1) output bins ----
            const float2* src = &yl[jj * kRowF2 + hh * kHalfF2];
#pragma unroll
            for (int q = 0; q < 32; ++q) {
                const float2 v = src[q];
                xr[q] = v.x;
                xi[q] = v.y;
            }
            __syncthreads();
        } else {
            // real parts first, then imaginary parts, through one float buffer of 32 rows
            float im_hold[kPass];              // imaginary outputs, stored after the real ones are read
#pragma unroll
            for (int pr = 0; pr < kPass / 2; ++pr) {
                const float2 A = acc[2 * pr], B = acc[2 * pr + 1];
                const auto sr = __builtin_amdgcn_permlane32_swap(__float_as_uint(A.x), __float_as_uint(B.x), false, false);
                const auto si = __builtin_amdgcn_permlane32_swap(__float_as_uint(A.y), __float_as_uint(B.y), false, false);
                const float r0r = __uint_as_float(sr[0]), r1r = __uint_as_float(sr[1]);
                const float r0i = __uint_as_float(si[0]), r1i = __uint_as_float(si[1]);
                const float dr = r0r - r1r, di = r0i - r1i;
                const int row = 2 * pr + (lane >> 5), q = lane & 31;
                ylds[row * kRowF1 + q] = r0r + r1r;
                ylds[row * kRowF1 + kHalfF1 + q] = dr * wcs + di * wsn;
                im_hold[2 * pr] = r0i + r1i;
                im_hold[2 * pr + 1] = di * wcs - dr * wsn;
            }
            __syncthreads();
            // lane (jj, hh) reads row jj, half hh: with rows of 72 floats and halves 36 apart,
            // any 16 lanes' 16-byte reads cover 64 distinct banks
            const float* src = &ylds[jj * kRowF1 + hh * kHalfF1];
#pragma unroll
            for (int q = 0; q < 32; ++q) xr[q] = src[q];
            __syncthreads();
#pragma unroll
            for (int pr = 0; pr < kPass / 2; ++pr) {
                const int row = 2 * pr + (lane >> 5), q = lane & 31;
                ylds[row * kRowF1 + q] = im_hold[2 * pr];
                ylds[row * kRowF1 + kHalfF1 + q] = im_hold[2 * pr + 1];
            }
            __syncthreads();
#pragma unroll
            for (int q = 0; q < 32; ++q) xi[q] = src[q];
            __syncthreads();
        }
        fft32(xr, xi);

        // ---- fine delay + bandpass, then write channel rows in ascending channel order ----
        // This lane holds channel c = 2q + hh (q = 0..31) of channel sample j; its phase in
        // cycles is f_c tau(j) = tau(j) (f_SB + (c - C/2) df), linear in q.  Exact phasors
        // (FP64 argument and reduction) every 4 steps of q, complex recurrence in between.
        const int j = jb + jj;
        const double tau = tau0 + (tau1 - tau0) * (double)j / (double)a.n_c;
        const double c1 = tau * a.df;                                  // cycles per channel
        // this lane's channels: c = 2 kW q + kW hh + wv (q = 0..31)
        const double c0 = fma((double)(kW * hh + wv - C / 2), c1, tau * fsb);   // cycles at q = 0
        const float2 step = phasor_rev(2.0 * kW * c1);                          // q -> q + 1
        float2 ph = make_float2(1.f, 0.f);
        const uint32_t lane_off = (uint32_t)(kW * hh + wv) * cstride + (uint32_t)(jb / kKBlock) * kbstride + (uint32_t)(jj * O_::kElem);
        const uint32_t lane_off_lo = lane_off + pstride;                // FP16-split lo plane
#pragma unroll
        for (int q = 0; q < 32; ++q) {
            if (q % 4 == 0) {
                ph = phasor_rev(fma((double)(2 * kW * q), c1, c0));
            } else {
                const float pr_ = ph.x * step.x - ph.y * step.y;
                ph.y = ph.x * step.y + ph.y * step.x;
                ph.x = pr_;
            }
            const int m = (q + 16) & 31;               // FFT bin 2m + hh is channel 2q + hh
            const int i = bitrev5(m);                  // register holding bin m
            const float b = blds[2 * kW * q + kW * hh + wv];   // bandpass x mode scale of channel c
            const float pr_ = ph.x * b, pi_ = ph.y * b;
            const float zr = xr[i] * pr_ - xi[i] * pi_;
            const float zi = xr[i] * pi_ + xi[i] * pr_;
            // the channel's base is wave-uniform (scalar adds); lane offsets are loop-invariant
            char* outq = out + (size_t)((uint32_t)(2 * kW * q) * cstride);
            char* dst = outq + lane_off;
            // non-temporal stores: the channelised data is written once here and read once by
            // the next kernel (measured 1-2 % faster than cached stores)
            if constexpr (OM == XM_FP32) {
                const float2v z2 = {zr, zi};
                __builtin_nontemporal_store(z2, (float2v*)dst);
            } else if constexpr (OM == XM_FP16_SPLIT) {
                // hi = fp16(z) (round to nearest even), lo = fp16(z - hi).  z - hi is exact in
                // FP32, so v_fma_mix{lo,hi}_f16 (z + 1 * (-hi) with hi read as fp16, result
                // rounded once to fp16) gives the same bits as converting hi back, subtracting
                // and converting, in one instruction per component.
                // Integer samples cannot overflow FP16 here: plan creation bounds the prescale
                // by the largest channel sample full-scale input can produce.  Float samples
                // have no such bound, so their components saturate at the largest FP16 value
                // instead of turning into infinities.
                float zr_ = zr, zi_ = zi;
                if constexpr (ST == ST_CF32) {
                    zr_ = __builtin_amdgcn_fmed3f(zr, -65504.f, 65504.f);
                    zi_ = __builtin_amdgcn_fmed3f(zi, -65504.f, 65504.f);
                }
                const float2v z2 = {zr_, zi_};
                const half2v hi = __builtin_convertvector(z2, half2v);
                const unsigned hb = __builtin_bit_cast(unsigned, hi);
                unsigned lb;
                asm("v_fma_mixlo_f16 %0, %1, 1.0, -%2 op_sel_hi:[0,0,1]" : "=v"(lb) : "v"(zr_), "v"(hb));
                asm("v_fma_mixhi_f16 %0, %1, 1.0, -%2 op_sel:[0,0,1] op_sel_hi:[0,0,1]" : "+v"(lb) : "v"(zi_), "v"(hb));
                __builtin_nontemporal_store(hb, (unsigned*)dst);
                __builtin_nontemporal_store(lb, (unsigned*)(outq + lane_off_lo));
            } else {
                const float qr = fminf(fmaxf(rintf(zr), -127.f), 127.f);
                const float qi = fminf(fmaxf(rintf(zi), -127.f), 127.f);
                const unsigned short v = (unsigned short)(((unsigned)(int)qr & 0xffu) | (((unsigned)(int)qi & 0xffu) << 8));
                __builtin_nontemporal_store(v, (unsigned short*)dst);
            }
            if (q % 4 == 3) __builtin_amdgcn_sched_barrier(0);   // bound live ranges per 4 channels
        }
    }
}

__global__ void zero_fill_kernel(uint4* p, int64_t n16, uint8_t* tail, int64_t ntail) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
    if (blockIdx.x == 0)
        for (int64_t i = threadIdx.x; i < ntail; i += blockDim.x) tail[i] = 0;
}

template <int ST, int C>
hipError_t launch_st(int x_mode, const FArgs& a, int n_streams, hipStream_t st) {
    const dim3 grid((unsigned)((int64_t)n_streams * a.n_chunks)), block(C);   // = SB * n_chunks * M
    switch (x_mode) {
        case XM_FP32: hipLaunchKernelGGL((fstage_kernel<ST, XM_FP32, C>), grid, block, 0, st, a); break;
        case XM_FP16_SPLIT: hipLaunchKernelGGL((fstage_kernel<ST, XM_FP16_SPLIT, C>), grid, block, 0, st, a); break;
        case XM_INT8: hipLaunchKernelGGL((fstage_kernel<ST, XM_INT8, C>), grid, block, 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int ST>
hipError_t launch_c(int x_mode, const FArgs& a, int n_streams, hipStream_t st) {
    switch (a.C) {
        case 64: return launch_st<ST, 64>(x_mode, a, n_streams, st);
        case 256: return launch_st<ST, 256>(x_mode, a, n_streams, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_fstage(int sample_type, int x_mode, const FArgs& a, int n_streams, hipStream_t st) {
    if (n_streams <= 0 || a.n_chunks <= 0) return hipSuccess;
    switch (sample_type) {
        case ST_CI8: return launch_c<ST_CI8>(x_mode, a, n_streams, st);
        case ST_CI16: return launch_c<ST_CI16>(x_mode, a, n_streams, st);
        case ST_CF32: return launch_c<ST_CF32>(x_mode, a, n_streams, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_zero_fill(void* p, int64_t bytes, hipStream_t st) {
    if (bytes <= 0) return hipSuccess;
    const int64_t n16 = ((uintptr_t)p % 16 == 0) ? bytes / 16 : 0;
    const int64_t ntail = bytes - n16 * 16;
    const int64_t blocks = n16 > 0 ? (n16 + 255) / 256 : 1;
    const unsigned g = (unsigned)(blocks < 4096 ? blocks : 4096);
    hipLaunchKernelGGL(zero_fill_kernel, dim3(g), dim3(256), 0, st, (uint4*)p, n16, (uint8_t*)p + n16 * 16, ntail);
    return hipGetLastError();
}

}  // namespace cobalt

// X stage of the FX correlator for gfx950: per channel, V = Z Z^H over all inputs
// (station x polarisation), integrated over the block ("Signal processing with GPU
// kernels", sec. 7.5: correlations of all pairs of antenna fields, averaged to ~1 s).
//
// MFMA form (FP16-split and int8): a complex Hermitian rank-K update written as two real
// contractions over K = 2 N_c interleaved (re, im) values:
//     Re V[a][b] = sum_k A[a][k] A[b][k]         (A = interleaved rows of Z)
//     Im V[a][b] = sum_k A[a][k] A'[b][k]        (A' = per sample (re, im) -> (-im, re))
// One workgroup owns one channel and keeps every lower-triangle 32x32 tile of V in
// accumulators; channel rows stream through LDS once.  An MFMA fragment of row block I
// (lane i: row 32I + i%32, 8 halves / 16 bytes of K) is simultaneously an A operand (row
// I) and a B operand (column I), so both operands of a tile come from the same LDS reads
// and the k order inside a fragment never matters.  A' is built in registers from the
// B-role fragments.
//   FP16-split: Z*2^k = hi + lo (two fp16 planes); V ~= hh + hl + lh accumulated in FP32
//   (the dropped lo*lo term is below 2^-22 of |Z|^2), scaled back by 2^-2k.  On a diagonal
//   tile (I = J) the lh product is the transpose of hl (real part) and minus its transpose
//   (imaginary part), so it is not multiplied but added from hl at the end (where registers
//   allow: every diagonal tile of the 152-input grid).
//   int8: exact int32 sums.
// Plain FP32 form: complex FMAs on the VALU over halves of 8x8 blocks of inputs, with partial
// sums over 128 channel samples folded into running totals.
#include <type_traits>

#include "cobalt_internal.h"

namespace cobalt {
namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef int intx16 __attribute__((ext_vector_type(16)));
typedef int intx4 __attribute__((ext_vector_type(4)));
typedef unsigned uintx4 __attribute__((ext_vector_type(4)));

template <int I, int N, class F>
__device__ __forceinline__ void static_for_impl(F& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for_impl<I + 1, N>(f);
    }
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) { static_for_impl<0, N>(f); }

// Lower-triangle tiles of an R x R block grid, column-major: (0,0),(1,0)..(R-1,0),(1,1)..
constexpr int tile_count(int R) { return R * (R + 1) / 2; }
constexpr int tile_J(int R, int idx) {
    int J = 0;
    while (idx >= R - J) { idx -= R - J; ++J; }
    return J;
}
constexpr int tile_I(int R, int idx) {
    int J = 0;
    while (idx >= R - J) { idx -= R - J; ++J; }
    return J + idx;
}
constexpr int kTilesPerWave = 4;
// blocks used by wave W as A (row) or B (column) operands
constexpr unsigned wave_blocks(int R, int W, bool as_b) {
    unsigned m = 0;
    for (int t = kTilesPerWave * W; t < kTilesPerWave * W + kTilesPerWave && t < tile_count(R); ++t)
        m |= 1u << (as_b ? tile_J(R, t) : tile_I(R, t));
    return m;
}

// Whether wave W of an R-block grid forms lh of its diagonal tiles from hl (FP16-split): each
// such tile holds one more accumulator pair, so only where at most 5 pairs fit in registers.
constexpr bool diag_from_hl(int R, int W) {
    int n = 0, d = 0;
    for (int t = kTilesPerWave * W; t < kTilesPerWave * W + kTilesPerWave && t < tile_count(R); ++t) {
        ++n;
        if (tile_I(R, t) == tile_J(R, t)) ++d;
    }
    return n + d <= 5;
}

template <int MODE> struct XCfg;
template <> struct XCfg<XM_FP16_SPLIT> {
    static constexpr int kKc = 32;            // complex samples per chunk (one K block)
    static constexpr int kSteps = 4;          // k-steps of 16 halves per chunk
    using acc_t = floatx16;
    using frag_t = half8;
};
template <> struct XCfg<XM_INT8> {
    static constexpr int kKc = 128;           // complex samples per chunk (four K blocks)
    static constexpr int kSteps = 8;          // k-steps of 32 bytes per chunk
    using acc_t = intx16;
    using frag_t = intx4;
};
constexpr int kRowB = 256;                    // LDS bytes per row and chunk (16 granules of 16 B)

// LDS rows are XOR-swizzled in 16-byte granules (granule g of row r is stored at g ^ (r%16)),
// so the 32 rows of one MFMA fragment read hit distinct banks without padding.
__device__ __forceinline__ int lds_off(int row, int g) { return row * kRowB + ((g ^ (row & 15)) << 4); }

// (re, im) -> (-im, re) on packed fp16 pairs
__device__ __forceinline__ uintx4 swapneg_f16(uintx4 d) {
    uintx4 r;
#pragma unroll
    for (int e = 0; e < 4; ++e) r[e] = __builtin_amdgcn_alignbit(d[e], d[e], 16) ^ 0x00008000u;
    return r;
}
// (re, im) -> (-im, re) on packed int8 pairs; inputs lie in [-127, 127]
__device__ __forceinline__ uintx4 swapneg_i8(uintx4 d) {
    uintx4 r;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const unsigned t = __builtin_amdgcn_perm(d[e], d[e], 0x02030001u);   // bytes (im, re) pairs
        const unsigned lo = t & 0x00ff00ffu;
        r[e] = (t & 0xff00ff00u) | ((0x01000100u - lo) & 0x00ff00ffu);
    }
    return r;
}

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// Issue the global -> LDS transfers of one chunk (rows < M) into LDS buffer `buf`.  One
// instruction moves 64 lanes x 16 B into 1 KB of consecutive LDS (4 rows); lane L of
// instruction i fills row 4i + L/16, stored granule L%16.  Rows >= M are never written.
//   FP16-split chunk = K block kb: [hi: M rows x 128 B][lo: M rows x 128 B]; logical granule
//   g < 8 is hi bytes 16g.., g >= 8 lo bytes 16(g-8)...
//   int8 chunk = K blocks kb..kb+3, each [M rows x 64 B]; logical granule g is block g/4,
//   bytes 16(g%4)...  Blocks past the last one are not loaded.
template <int MODE>
__device__ __forceinline__ void issue_chunk(const XArgs& a, const char* __restrict__ chan, char* buf, int kc0, int wave, int lane) {
    const int n_inst = (a.M + 3) / 4;
    const int rsub = lane >> 4, p = lane & 15;
    for (int i = wave; i < n_inst; i += 4) {
        const int row = 4 * i + rsub;
        const int g = p ^ (row & 15);
        const char* src;
        bool ok = row < a.M;
        if constexpr (MODE == XM_FP16_SPLIT) {
            const char* blk = chan + (int64_t)(kc0 / kKBlock) * (2 * a.M * 128);
            src = blk + (g >> 3) * (a.M * 128) + row * 128 + (g & 7) * 16;
        } else {
            const int kb = kc0 / kKBlock + (g >> 2);
            ok = ok && kb < a.n_kb;
            src = chan + (int64_t)kb * (a.M * 64) + row * 64 + (g & 3) * 16;
        }
        // non-temporal: each byte of the channelised data is read once (measured ~1.5 % faster)
        if (ok) __builtin_amdgcn_global_load_lds((const void*)src, (lds_ptr_t)(buf + i * 1024), 16, 0, 2);
    }
}

// Zero the LDS entries of columns >= N_c (the last, partial chunk) and of K blocks that were
// not loaded, for rows < M.
template <int MODE>
__device__ __forceinline__ void zero_tail(const XArgs& a, char* buf, int kc0, int tid) {
    constexpr int kKc = XCfg<MODE>::kKc;
    const int first = a.n_c - kc0;                     // first column to clear
    const int cols = kKc - first;
    for (int id = tid; id < a.M * cols; id += 256) {
        const int row = id / cols, c = first + id % cols;
        if constexpr (MODE == XM_FP16_SPLIT) {
            *(unsigned*)(buf + lds_off(row, c >> 2) + (c & 3) * 4) = 0u;        // hi
            *(unsigned*)(buf + lds_off(row, 8 + (c >> 2)) + (c & 3) * 4) = 0u;  // lo
        } else {
            *(unsigned short*)(buf + lds_off(row, c >> 3) + (c & 7) * 2) = 0;
        }
    }
}

template <int MODE, int R, int W>
__device__ __forceinline__ void xwave(const XArgs& a, const char* __restrict__ chan, char* lds, int tid) {
    using C_ = XCfg<MODE>;
    using acc_t = typename C_::acc_t;
    using frag_t = typename C_::frag_t;
    constexpr int NT = tile_count(R);
    constexpr int T0 = kTilesPerWave * W;
    constexpr int NW = NT - T0 <= 0 ? 0 : (NT - T0 > kTilesPerWave ? kTilesPerWave : NT - T0);
    constexpr unsigned useA = wave_blocks(R, W, false) | wave_blocks(R, W, true);
    constexpr unsigned useB = wave_blocks(R, W, true);
    constexpr bool kDiagHl = MODE == XM_FP16_SPLIT && diag_from_hl(R, W);
    constexpr int kBufB = R * 32 * kRowB;
    const int lane = tid & 63;

    acc_t vre[kTilesPerWave], vim[kTilesPerWave];
    acc_t xre[kTilesPerWave], xim[kTilesPerWave];     // hl of diagonal tiles (FP16-split)
#pragma unroll
    for (int t = 0; t < kTilesPerWave; ++t) {
        vre[t] = acc_t{};
        vim[t] = acc_t{};
        xre[t] = acc_t{};
        xim[t] = acc_t{};
    }

    // rows M .. 32R-1 stay zero in both buffers
    for (int off = a.M * kRowB + tid * 16; off < kBufB; off += 256 * 16) {
        *(uint4*)(lds + off) = make_uint4(0, 0, 0, 0);
        *(uint4*)(lds + kBufB + off) = make_uint4(0, 0, 0, 0);
    }
    __syncthreads();
    if (a.n_c > 0) issue_chunk<MODE>(a, chan, lds, 0, W, lane);

    int cur = 0;
    for (int kc0 = 0; kc0 < a.n_c; kc0 += C_::kKc) {
        char* buf = lds + cur * kBufB;
        __builtin_amdgcn_s_waitcnt(0);        // this wave's transfers of chunk kc0 have landed
        __syncthreads();                      // ... and everyone's; the other buffer is free
        if (kc0 + C_::kKc < a.n_c) issue_chunk<MODE>(a, chan, lds + (cur ^ 1) * kBufB, kc0 + C_::kKc, W, lane);
        if (kc0 + C_::kKc > a.n_c) {          // last, partial chunk (uniform)
            zero_tail<MODE>(a, buf, kc0, tid);
            __syncthreads();
        }
        if constexpr (NW > 0) {
#pragma unroll
            for (int ks = 0; ks < C_::kSteps; ++ks) {
                const int row = lane & 31;
                const int g = 2 * ks + (lane >> 5);
                if constexpr (MODE == XM_FP16_SPLIT) {
                    uintx4 fh[R], fl[R], gh[R], gl[R];
                    static_for<R>([&](auto bi) {
                        constexpr int b = decltype(bi)::value;
                        if constexpr ((useA >> b) & 1u) {
                            fh[b] = *(const uintx4*)(buf + lds_off(32 * b + row, g));
                            fl[b] = *(const uintx4*)(buf + lds_off(32 * b + row, 8 + g));
                        }
                        if constexpr ((useB >> b) & 1u) {
                            gh[b] = swapneg_f16(fh[b]);
                            gl[b] = swapneg_f16(fl[b]);
                        }
                    });
                    // three products (hh, hl, lh), each over all tiles: independent accumulators
                    // between dependent MFMAs; diagonal tiles keep hl apart and skip lh
                    static_for<3>([&](auto pi) {
                        constexpr int pr = decltype(pi)::value;
                        static_for<NW>([&](auto ti) {
                            constexpr int t = decltype(ti)::value;
                            constexpr int I = tile_I(R, T0 + t), J = tile_J(R, T0 + t);
                            constexpr bool dg = kDiagHl && I == J;
                            if constexpr (!(dg && pr == 2)) {
                                const frag_t A = __builtin_bit_cast(frag_t, pr == 2 ? fl[I] : fh[I]);
                                const frag_t B = __builtin_bit_cast(frag_t, pr == 1 ? fl[J] : fh[J]);
                                const frag_t Bs = __builtin_bit_cast(frag_t, pr == 1 ? gl[J] : gh[J]);
                                if constexpr (dg && pr == 1) {
                                    xre[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A, B, xre[t], 0, 0, 0);
                                    xim[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A, Bs, xim[t], 0, 0, 0);
                                } else {
                                    vre[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A, B, vre[t], 0, 0, 0);
                                    vim[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(A, Bs, vim[t], 0, 0, 0);
                                }
                            }
                        });
                    });
                } else {
                    uintx4 f[R], gg[R];
                    static_for<R>([&](auto bi) {
                        constexpr int b = decltype(bi)::value;
                        if constexpr ((useA >> b) & 1u) f[b] = *(const uintx4*)(buf + lds_off(32 * b + row, g));
                        if constexpr ((useB >> b) & 1u) gg[b] = swapneg_i8(f[b]);
                    });
                    static_for<NW>([&](auto ti) {
                        constexpr int t = decltype(ti)::value;
                        constexpr int I = tile_I(R, T0 + t), J = tile_J(R, T0 + t);
                        const frag_t A = __builtin_bit_cast(frag_t, f[I]);
                        const frag_t B = __builtin_bit_cast(frag_t, f[J]);
                        const frag_t Bs = __builtin_bit_cast(frag_t, gg[J]);
                        vre[t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, B, vre[t], 0, 0, 0);
                        vim[t] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A, Bs, vim[t], 0, 0, 0);
                    });
                }
            }
        }
        cur ^= 1;
    }

    // ---- diagonal tiles (FP16-split): Re += hl + hl^T, Im += hl - hl^T, through LDS ----
    if constexpr (MODE == XM_FP16_SPLIT) {
        __syncthreads();                      // every wave is done with the chunk buffers
        constexpr int kTw = 2 * 32 * 33;      // floats per wave: two padded 32 x 32 tiles
        float* tr = (float*)lds + W * kTw;
        static_for<NW>([&](auto ti) {
            constexpr int t = decltype(ti)::value;
            constexpr int I = tile_I(R, T0 + t), J = tile_J(R, T0 + t);
            if constexpr (kDiagHl && I == J) {
                static_assert((W + 1) * kTw * 4 <= 2 * R * 32 * kRowB, "transpose area inside LDS");
                const int col = lane & 31;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    tr[row * 33 + col] = xre[t][r];
                    tr[32 * 33 + row * 33 + col] = xim[t][r];
                }
                // the same wave reads the transpose back (its LDS operations complete in order)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                    vre[t][r] += xre[t][r] + tr[col * 33 + row];
                    vim[t][r] += xim[t][r] - tr[32 * 33 + col * 33 + row];
                }
            }
        });
    }

    // ---- epilogue: stored baselines s1 >= s2, all four polarisation products ----
    if constexpr (NW > 0) {
        const int64_t ch = blockIdx.x;
        const int64_t B = (int64_t)a.S * (a.S + 1) / 2;
        static_for<NW>([&](auto ti) {
            constexpr int t = decltype(ti)::value;
            constexpr int I = tile_I(R, T0 + t), J = tile_J(R, T0 + t);
            const int b = 32 * J + (lane & 31);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int aa = 32 * I + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                if (aa < a.M && b < a.M) {
                    const int s1 = aa >> 1, s2 = b >> 1;
                    if (s1 >= s2) {
                        const int64_t idx = (ch * B + (int64_t)s1 * (s1 + 1) / 2 + s2) * 4 + 2 * (aa & 1) + (b & 1);
                        if constexpr (MODE == XM_FP16_SPLIT) {
                            const float re = vre[t][r] * a.out_scale;
                            const float im = aa == b ? 0.f : vim[t][r] * a.out_scale;
                            ((float2*)a.vis)[idx] = make_float2(re, im);
                        } else {
                            ((int2*)a.vis)[idx] = make_int2(vre[t][r], aa == b ? 0 : vim[t][r]);
                        }
                    }
                }
            }
        });
    }
}

template <int MODE, int R>
__global__ __launch_bounds__(256, 2) void xstage_mfma_kernel(XArgs a) {
    __shared__ __attribute__((aligned(1024))) char lds[2 * R * 32 * kRowB];   // two chunk buffers
    const int tid = threadIdx.x;
    const char* chan = (const char*)a.chan + (int64_t)blockIdx.x * a.chan_stride;
    switch (tid >> 6) {
        case 0: xwave<MODE, R, 0>(a, chan, lds, tid); break;
        case 1: xwave<MODE, R, 1>(a, chan, lds, tid); break;
        case 2: xwave<MODE, R, 2>(a, chan, lds, tid); break;
        default: xwave<MODE, R, 3>(a, chan, lds, tid); break;
    }
}

template <int MODE>
hipError_t launch_mode(const XArgs& a, hipStream_t st) {
    const int R = (a.M + 31) / 32;
    const dim3 grid((unsigned)a.n_chan), block(256);
    switch (R) {
        case 1: hipLaunchKernelGGL((xstage_mfma_kernel<MODE, 1>), grid, block, 0, st, a); break;
        case 2: hipLaunchKernelGGL((xstage_mfma_kernel<MODE, 2>), grid, block, 0, st, a); break;
        case 3: hipLaunchKernelGGL((xstage_mfma_kernel<MODE, 3>), grid, block, 0, st, a); break;
        case 4: hipLaunchKernelGGL((xstage_mfma_kernel<MODE, 4>), grid, block, 0, st, a); break;
        case 5: hipLaunchKernelGGL((xstage_mfma_kernel<MODE, 5>), grid, block, 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ plain FP32 form ---
constexpr int kF32Kc = 16;        // complex samples per LDS chunk
// Blocked accumulation: products are summed over kF32Fold channel samples into partial sums,
// which are then added to the running totals.  A single running sum over all N_c samples
// leaves a relative rounding error of about u sqrt(N_c) / 6 (u = 2^-24; the additions round
// at the size of the growing sum); partial sums of b samples folded into the totals leave
// about u (b / sqrt(N_c) + sqrt(N_c / b)) / 6, smallest near b = sqrt(N_c): 7.7 times less
// at N_c = 3072 and b = 128.
constexpr int kF32Fold = 128;
static_assert(kF32Fold % kF32Kc == 0, "a fold spans whole LDS chunks");

// One thread per half (4 rows x 8 columns) of an 8x8 block of inputs in the lower triangle;
// complex FMAs from an LDS-staged chunk of kF32Kc channel samples.  The half-block keeps the
// partial sums and the running totals in registers at three waves per SIMD; the kernel
// stays bound by its FMAs (per chunk step a wave issues 128 FMAs against 12 LDS reads).  A
// workgroup of up to kF32Threads threads covers a whole channel (every input row staged
// once) up to 190 blocks (152 inputs).
constexpr int kF32Threads = 512;
__global__ __launch_bounds__(kF32Threads) void xstage_fp32_kernel(XArgs a) {
    // [kF32Kc][ls] complex samples, row r of input at r + r/16: across the lanes of a wave the
    // 16 distinct (row block, half) operands of a read land in distinct bank pairs
    extern __shared__ float2 zl[];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int nhalf = a.n_blocks8 * (a.n_blocks8 + 1);   // two halves per lower-triangle block
    const int groups = (nhalf + nthr - 1) / nthr;
    const int64_t ch = blockIdx.x / groups;
    const int g = blockIdx.x % groups;
    const int rows = 8 * a.n_blocks8, ls = rows + rows / 16 + 1;
    const float2* __restrict__ z = (const float2*)((const char*)a.chan + ch * a.chan_stride);

    // this thread's 8x8 block (A >= Bk) in the lower triangle of block rows, and its half
    const int hb = g * nthr + tid;
    const bool active = hb < nhalf;
    const int blk = hb >> 1, half = hb & 1;
    int A = 0, Bk = 0;
    if (active) {
        A = (int)((sqrtf(8.f * blk + 1.f) - 1.f) * 0.5f);
        while (A * (A + 1) / 2 > blk) --A;
        while ((A + 1) * (A + 2) / 2 <= blk) ++A;
        Bk = blk - A * (A + 1) / 2;
    }
    const int ra = 8 * A + 4 * half;               // first row of this half
    float vr[4][8], vi[4][8];           // partial sums of the current fold
    float tr[4][8], ti[4][8];           // running totals
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) { vr[i][j] = 0.f; vi[i][j] = 0.f; tr[i][j] = 0.f; ti[i][j] = 0.f; }

    for (int kc0 = 0; kc0 < a.n_c; kc0 += kF32Kc) {
        if (kc0 % kF32Fold == 0 && kc0 > 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    tr[i][j] += vr[i][j];
                    ti[i][j] += vi[i][j];
                    vr[i][j] = 0.f;
                    vi[i][j] = 0.f;
                }
        }
        __syncthreads();
        for (int id = tid; id < rows * kF32Kc; id += nthr) {
            const int row = id / kF32Kc, k = id % kF32Kc, col = kc0 + k;
            float2 v = make_float2(0.f, 0.f);
            if (row < a.M && col < a.n_c) v = z[((int64_t)(col / kKBlock) * a.M + row) * kKBlock + (col % kKBlock)];
            zl[k * ls + row + (row >> 4)] = v;
        }
        __syncthreads();
        if (active) {
            for (int k = 0; k < kF32Kc; ++k) {
                float2 xa[4], xb[8];
#pragma unroll
                for (int i = 0; i < 4; ++i) xa[i] = zl[k * ls + ra + i + ((ra + i) >> 4)];
#pragma unroll
                for (int j = 0; j < 8; ++j) xb[j] = zl[k * ls + 8 * Bk + j + ((8 * Bk + j) >> 4)];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        vr[i][j] = fmaf(xa[i].x, xb[j].x, fmaf(xa[i].y, xb[j].y, vr[i][j]));
                        vi[i][j] = fmaf(xa[i].y, xb[j].x, fmaf(-xa[i].x, xb[j].y, vi[i][j]));
                    }
            }
        }
    }
    if (!active) return;
    const int64_t B = (int64_t)a.S * (a.S + 1) / 2;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int aa = ra + i, b = 8 * Bk + j;
            if (aa < a.M && b < a.M && (aa >> 1) >= (b >> 1)) {
                const int s1 = aa >> 1, s2 = b >> 1;
                const int64_t idx = (ch * B + (int64_t)s1 * (s1 + 1) / 2 + s2) * 4 + 2 * (aa & 1) + (b & 1);
                ((float2*)a.vis)[idx] = make_float2(tr[i][j] + vr[i][j], aa == b ? 0.f : ti[i][j] + vi[i][j]);
            }
        }
}

}  // namespace

hipError_t launch_xstage_mfma(int x_mode, const XArgs& a, hipStream_t st) {
    if (a.n_chan <= 0) return hipSuccess;
    if (x_mode == XM_FP16_SPLIT) return launch_mode<XM_FP16_SPLIT>(a, st);
    if (x_mode == XM_INT8) return launch_mode<XM_INT8>(a, st);
    return hipErrorInvalidValue;
}

hipError_t launch_xstage_fp32(const XArgs& a, hipStream_t st) {
    if (a.n_chan <= 0) return hipSuccess;
    const int nhalf = a.n_blocks8 * (a.n_blocks8 + 1);
    const int nthr = nhalf < kF32Threads ? (nhalf + 63) / 64 * 64 : kF32Threads;
    const int groups = (nhalf + nthr - 1) / nthr;
    const size_t lds = (size_t)kF32Kc * (8 * a.n_blocks8 + (8 * a.n_blocks8) / 16 + 1) * sizeof(float2);
    hipLaunchKernelGGL(xstage_fp32_kernel, dim3((unsigned)((int64_t)a.n_chan * groups)), dim3(nthr), lds, st, a);
    return hipGetLastError();
}

}  // namespace cobalt

// Lost-sample flags: which channel samples read a lost input sample, and per-baseline
// weights (channel samples valid for both stations).
//
// Lost or late input is recorded and travels with the data product ("Processing steps",
// sec. 3.2; "Dealing with jitter and hardware failure", sec. 7.2).  Channel sample j of a
// stream is the FIR output over input rows j-T+1 .. j of C samples each (rows before the
// block come from the previous block), so it is flagged when any of those T rows holds a
// lost sample.  The F stage writes flagged channel samples as zero, so they drop out of every
// visibility, and the weights count what remains per baseline.
//
// Bit conventions: row word w of a stream holds rows 32w .. 32w+31 (bit i = row 32w+i); the
// carried history word holds rows -15 .. -1 in bits 17 .. 31, i.e. it is row word -1.  Then
// channel word w = bits 32 .. 63 of  OR_{d<16} (x << d)  with  x = (row word w) << 32 | (row
// word w-1).
#include "cobalt_internal.h"

namespace cobalt {
namespace {

static_assert(kHistRows == 15, "history bits 17..31 of the previous row word");

// One wave per (station, subband): lanes take 64 consecutive row words at a time; the
// neighbour's row word comes from the lane below (the previous iteration's last lane, or the
// carried history, for lane 0).
__global__ __launch_bounds__(64) void chanflag_kernel(FlagArgs a) {
    const int lane = threadIdx.x;
    const int64_t sst = blockIdx.x;                       // s * SB + sb
    const int s = (int)(sst / a.SB);
    const uint32_t* __restrict__ fl = a.flags ? a.flags + sst * a.flag_words : nullptr;
    const int64_t g = a.coarse ? a.coarse[s] : 0;         // window start in the row
    const int b = (int)(g & 31);
    const uint32_t lowmask = b ? (1u << b) - 1u : 0u;
    uint32_t carry = a.hist_old[sst];
    uint32_t* __restrict__ out = a.cflag + sst * a.n_words;
    const int wl = (a.n_c - 1) >> 5;                       // row word holding the last row
    const int wr = a.C >> 5;                               // flag words per row of C samples
    for (int w0 = 0; w0 < a.n_words; w0 += 64) {
        const int w = w0 + lane;
        uint32_t rw = 0;
        if (fl && w < a.n_words) {
            // rows r = 32w + i cover samples g + Cr .. g + Cr + C-1 of the row: bits b..31 of
            // word i0, all of words i0+1 .. i0+C/32-1 and bits 0..b-1 of word i0+C/32 (present
            // when b > 0, since the window ends inside the row)
            const int rmax = min(32, a.n_c - 32 * w);
            const int64_t base = (g >> 5) + (int64_t)w * 32 * wr;
            for (int i = 0; i < rmax; ++i) {
                const int64_t i0 = base + (int64_t)wr * i;
                uint32_t any = fl[i0] >> b;
                for (int k = 1; k < wr; ++k) any |= fl[i0 + k];
                if (b) any |= fl[i0 + wr] & lowmask;
                rw |= (any != 0u ? 1u : 0u) << i;
            }
        }
        uint32_t prev = (uint32_t)__shfl_up((int)rw, 1, 64);
        if (lane == 0) prev = carry;
        const uint64_t x = ((uint64_t)rw << 32) | prev;
        uint64_t y = x | (x << 1);
        y |= y << 2;
        y |= y << 4;
        y |= y << 8;                                        // OR over shifts 0 .. 15
        if (w < a.n_words) {
            uint32_t cw = (uint32_t)(y >> 32);
            const int left = a.n_c - 32 * w;                // >= 1 for every word of the pitch
            if (left < 32) cw &= (1u << left) - 1u;
            out[w] = cw;
        }
        if (w == wl) {
            // rows n_c-15 .. n_c-1 are bits e-14 .. e of x, e = 32 + (n_c-1) % 32
            const int e = 32 + ((a.n_c - 1) & 31);
            a.hist_new[sst] = (uint32_t)((x >> (e - 14)) & 0x7fffu) << 17;
        }
        carry = (uint32_t)__shfl((int)rw, 63, 64);
    }
}

// One thread per (subband, baseline): popcount of the channel samples valid for both
// stations.  Without flags every baseline has all N_c.
__global__ __launch_bounds__(256) void weights_kernel(const uint32_t* __restrict__ cflag, int32_t* __restrict__ weights,
                                                      int S, int SB, int n_c, int n_words) {
    const int B = S * (S + 1) / 2;
    const int bl = blockIdx.x * 256 + threadIdx.x;
    const int sb = blockIdx.y;
    if (bl >= B) return;
    if (!cflag) {
        weights[(int64_t)sb * B + bl] = n_c;
        return;
    }
    int s1 = (int)((sqrtf(8.f * bl + 1.f) - 1.f) * 0.5f);
    while (s1 * (s1 + 1) / 2 > bl) --s1;
    while ((s1 + 1) * (s1 + 2) / 2 <= bl) ++s1;
    const int s2 = bl - s1 * (s1 + 1) / 2;
    const uint32_t* f1 = cflag + ((int64_t)s1 * SB + sb) * n_words;
    const uint32_t* f2 = cflag + ((int64_t)s2 * SB + sb) * n_words;
    int cnt = 0;
    for (int w = 0; w < n_words; ++w) {
        const int left = n_c - 32 * w;
        const uint32_t valid = left >= 32 ? 0xffffffffu : (1u << left) - 1u;
        cnt += __popc(~(f1[w] | f2[w]) & valid);
    }
    weights[(int64_t)sb * B + bl] = cnt;
}

}  // namespace

hipError_t launch_chanflags(const FlagArgs& a, hipStream_t st) {
    if (a.n_c == 0) return hipSuccess;
    hipLaunchKernelGGL(chanflag_kernel, dim3((unsigned)((int64_t)a.S * a.SB)), dim3(64), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_weights(const uint32_t* cflag, int32_t* weights, int S, int SB, int n_c, int n_words, hipStream_t st) {
    const int B = S * (S + 1) / 2;
    hipLaunchKernelGGL(weights_kernel, dim3((unsigned)((B + 255) / 256), (unsigned)SB), dim3(256), 0, st, cflag, weights, S, SB,
                       n_c, n_words);
    return hipGetLastError();
}

}  // namespace cobalt

// Internal declarations shared by the plan (C ABI) and the kernels of libcobalt.so.
// Not installed; the public interface is include/cobalt.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cobalt {

// Built instantiation: C = 64 channels, T = 16 taps (the paper's 64-channel correlator
// setting with a 16-tap polyphase FIR).
constexpr int kC = 64;
constexpr int kT = 16;
constexpr int kHistRows = kT - 1;              // FIR history in rows of C samples
constexpr int kHist = kHistRows * kC;          // 960 samples carried per input stream
constexpr int kKBlock = 32;                    // channel samples per K block of the channelised layout
constexpr int kPitchAlign = kKBlock;           // channelised rows padded to whole K blocks
constexpr int kMaxMfmaInputs = 160;            // 5 row blocks of 32 (80 stations)
constexpr int kMaxFp32Inputs = 256;
constexpr int kFChunk = 256;                  // channel samples per F-stage workgroup

enum SampleType { ST_CI8 = 1, ST_CI16 = 2, ST_CF32 = 3 };
enum XMode { XM_FP32 = 0, XM_FP16_SPLIT = 1, XM_INT8 = 2 };

struct FArgs {
    const void* in;          // [S][P][SB][N] samples
    const void* hist_old;    // [S*P*SB][kHist] samples, stream order (s*P + p)*SB + sb
    void* hist_new;          // same layout, written by the last chunk of each stream
    void* out;               // channelised buffer, K-blocked (see cobalt.h)
    const float* fir;        // [kT * kC]
    const float* bscale;     // [kC] bandpass * mode scale (2^k or requant gain)
    const double* f_sb;      // [SB] subband sky centre frequency (Hz)
    const double* delays;    // [S][2] residual delay (s) at block start / end
    int64_t N;               // samples per block per stream
    int32_t S, SB, M, n_c, pitch, n_chunks, n_kb;
    double df;               // channel width f_s / C (Hz)
};

struct XArgs {
    const void* chan;        // channelised buffer
    void* vis;               // [SB*C][B][4] complex
    int64_t chan_stride;     // bytes per channel in the channelised buffer
    int32_t M, S, n_c, pitch, n_chan, n_blocks8, n_kb;
    float out_scale;         // FP16-split: 2^-2k
};

// Launchers (return the hipError_t of the launch).
hipError_t launch_fstage(int sample_type, int x_mode, const FArgs& a, int n_streams, hipStream_t st);
hipError_t launch_xstage_mfma(int x_mode, const XArgs& a, hipStream_t st);
hipError_t launch_xstage_fp32(const XArgs& a, hipStream_t st);
hipError_t launch_zero_fill(void* p, int64_t bytes, hipStream_t st);
hipError_t launch_device_copy(void* dst, const void* src, int64_t bytes, hipStream_t st);
hipError_t launch_apply_gains(const void* vis0, const void* gains, void* vis, int n_chan, int S, hipStream_t st);
hipError_t launch_apply_gains_adjoint(const void* vis0, const void* gains, const void* grad_vis, void* grad_gains, int n_chan,
                                      int S, hipStream_t st);

}  // namespace cobalt

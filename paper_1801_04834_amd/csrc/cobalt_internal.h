// Internal declarations shared by the plan (C ABI) and the kernels of libcobalt.so.
// Not installed; the public interface is include/cobalt.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cobalt.h"

namespace cobalt {

// Built instantiations: C = 64 channels (the correlator setting) and C = 256 (the paper's
// beamformer front end and the correlator's finest resolution), T = 16 taps.
constexpr int kT = 16;
constexpr int kHistRows = kT - 1;              // FIR history in rows of C samples
constexpr int kKBlock = 32;                    // channel samples per K block of the channelised layout
constexpr int kPitchAlign = kKBlock;           // channelised rows padded to whole K blocks
constexpr int kMaxMfmaInputs = 160;            // 5 row blocks of 32 (80 stations)
constexpr int kMaxFp32Inputs = 256;
constexpr int kFChunk = 256;                  // channel samples per F-stage workgroup

enum SampleType { ST_CI8 = 1, ST_CI16 = 2, ST_CF32 = 3 };
enum XMode { XM_FP32 = 0, XM_FP16_SPLIT = 1, XM_INT8 = 2 };

struct FArgs {
    const void* in;          // [S][P][SB][row_len] samples; the block window starts at coarse[s]
    const void* hist_old;    // [S*P*SB][kHistRows*C] samples, stream order (s*P + p)*SB + sb
    void* hist_new;          // same layout, written by the last chunk of each stream
    void* out;               // channelised buffer, K-blocked (see cobalt.h)
    const float* fir;        // [kT * C]
    const float* bscale;     // [C] bandpass * mode scale (2^k or requant gain)
    const double* f_sb;      // [SB] subband sky centre frequency (Hz)
    const double* delays;    // [S][2] residual delay (s) at block start / end
    const int32_t* coarse;   // [S] window start of each station in its rows, or null (0)
    const uint32_t* cflag;   // [S*SB][n_words] flagged channel samples (bit j%32 of word j/32), or null
    int64_t N;               // samples per block window per stream
    int64_t row_len;         // samples per input row (N + guard)
    int32_t C;               // channels: 64 or 256
    int32_t S, SB, M, n_c, pitch, n_chunks, n_kb, n_words;
    double df;               // channel width f_s / C (Hz)
};

// Lost-sample flags -> flagged channel samples (FIR window rule) and the row flags carried
// to the next block.
struct FlagArgs {
    const uint32_t* flags;   // [S][SB][flag_words] lost-sample bits of the input rows, or null
    int64_t flag_words;
    const int32_t* coarse;   // [S] or null
    const uint32_t* hist_old;// [S*SB] flags of the kHistRows rows before the block, bits 17..31
    uint32_t* hist_new;      // same, for the next block
    uint32_t* cflag;         // [S*SB][n_words]
    int32_t S, SB, n_c, n_words;
    int32_t C;               // samples per row (channels): a multiple of 32
};

struct XArgs {
    const void* chan;        // channelised buffer
    void* vis;               // [SB*C][B][4] complex
    int64_t chan_stride;     // bytes per channel in the channelised buffer
    int32_t M, S, n_c, pitch, n_chan, n_blocks8, n_kb;
    float out_scale;         // FP16-split: 2^-2k
};

// Beamformer over an FP16-split channelised buffer.
struct BeamArgs {
    const void* chan;        // channelised buffer (FP16-split planes, K-blocked)
    int64_t chan_stride;     // bytes per channel
    const double* f_sb;      // [SB] subband sky centre frequency (Hz)
    const double* dtau;      // [NB][S] beam delay offsets (s), device
    void* coherent;          // [SB*C][N_c/n_int][n_stokes][NB] float, or null
    void* voltages;          // [SB*C][N_c][P][vstride] float (re, im), or null
    void* incoherent;        // [SB*C][N_c/n_int][n_stokes] float, or null
    double df;               // channel width (Hz)
    int32_t C, S, NB, n_c, n_kb, n_chan, n_int, n_stokes;
    int32_t vstride;         // beams per voltage row (>= NB)
    float vscale;            // 2^-k: undoes the FP16-split prescale
};

// Output-resolution transform of beamformed voltages (256 channels -> c_out channels).
struct TfArgs {
    const void* vin;         // [SB][256][N_c][P][vstride] float (re, im): the beamformer's voltages
    void* vout;              // [SB][N_c 256 / c_out][c_out][P][vstride] float (re, im), or null
    void* sout;              // [SB][N_c 256 / c_out / n_int][c_out][n_stokes][NB] float, or null
    int32_t SB, n_c, NB, n_bg, c_out, n_stokes, n_int;
    int32_t vstride;         // beams per voltage row (>= NB)
};

// Launchers (return the hipError_t of the launch).
hipError_t launch_fstage(int sample_type, int x_mode, const FArgs& a, int n_streams, hipStream_t st);
hipError_t launch_xstage_mfma(int x_mode, const XArgs& a, hipStream_t st);
hipError_t launch_xstage_fp32(const XArgs& a, hipStream_t st);
hipError_t launch_chanflags(const FlagArgs& a, hipStream_t st);
hipError_t launch_weights(const uint32_t* cflag, int32_t* weights, int S, int SB, int n_c, int n_words, hipStream_t st);
hipError_t launch_beamformer(const BeamArgs& a, hipStream_t st);
hipError_t launch_beam_transform(const TfArgs& a, hipStream_t st);
hipError_t launch_zero_fill(void* p, int64_t bytes, hipStream_t st);
hipError_t launch_device_copy(void* dst, const void* src, int64_t bytes, hipStream_t st);
hipError_t launch_mfma_probe(int x_mode, int64_t iters, int workgroups, float* sink, hipStream_t st);
hipError_t launch_device_fanout(void* dst0, void* dst1, const void* src, int64_t bytes, hipStream_t st);
hipError_t launch_apply_gains(const void* vis0, const void* gains, void* vis, int n_chan, int S, hipStream_t st);
hipError_t launch_apply_gains_adjoint(const void* vis0, const void* gains, const void* grad_vis, void* grad_gains, int n_chan,
                                      int S, hipStream_t st);

// cobalt_plan_create with the device workspace given by the caller (d_workspace: 256-byte
// aligned, cobalt_estimate_bytes() bytes, left allocated by cobalt_plan_destroy) or, for
// NULL, allocated by the plan.  Used by the streaming service, which carves observation
// workspaces out of one arena allocated at its creation.
int plan_create_impl(const cobalt_config* cfg, void* d_workspace, cobalt_plan** out);

}  // namespace cobalt

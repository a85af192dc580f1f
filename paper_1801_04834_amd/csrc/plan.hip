// C ABI of libcobalt.so (declared in include/cobalt.h): plan validation, device workspace,
// FIR history, per-call delay staging and kernel launches.
//
// The paper wraps every GPU kernel in a class that owns its launch configuration and
// buffer sizes and documents which buffers each kernel reads and writes ("Signal
// processing with GPU kernels", sec. 7.5); it allocates buffers once at initialisation
// and keeps a few device buffers that kernels alternate between (sec. 7.1, sec. 7.5).
// Here the plan plays that role: one allocation at create, the two FIR-history buffers
// alternate between blocks, and observation constants are fixed at create.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "../../include/cobalt.h"
#include "cobalt_internal.h"

using namespace cobalt;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

constexpr int kRing = 8;   // delay staging slots (pinned host + device)

struct Sizes {
    int64_t S, P, SB, C, T, N, n_c, pitch, M, B, streams;
    int64_t sample_bytes, input_bytes, chan_elem_bytes, chan_planes, chan_stride, chan_bytes, vis_bytes;
    int64_t hist_bytes, table_bytes, workspace_bytes;
    int64_t n_words, cflag_bytes, rowhist_bytes, stage_bytes;
};

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Largest power-of-two prescale k for which no channelised value of an integer sample type
// can overflow FP16.  Integer samples are converted to float exactly (sec. 3.2), so every
// component of a channel sample is bounded by the triangle inequality through the chain:
//   |Z| = |b_c| |X_k| <= max|b| sum_p |y_j[p]| <= max|b| sum_m |h[m]| max|x|,
// with max|x| = 2^15 sqrt(2) (int16) or 2^7 sqrt(2) (int8) for the complex sample
// (-2^15, -2^15) resp. (-2^7, -2^7); the delay phasor has unit modulus.  A sign-matched
// input (x = sgn(h) (1 + i) 2^15 over one FIR window) reaches the bound in the channel of
// FFT bin 0.  FP16 round-to-nearest overflows at 65520; the 2^-10 margin covers the F
// stage's FP32 rounding on the way.  Returns INT32_MIN when the sample type has no bound
// (float samples).
int fp16_prescale_limit(const cobalt_config* c) {
    if (c->sample_type == COBALT_CF32) return INT32_MIN;
    double sh = 0.0;
    for (int i = 0; i < c->n_taps * c->n_channels; ++i) sh += std::fabs((double)c->h_fir[i]);
    double bmax = 1.0;
    if (c->h_bandpass) {
        bmax = 0.0;
        for (int i = 0; i < c->n_channels; ++i) bmax = std::fmax(bmax, std::fabs((double)c->h_bandpass[i]));
    }
    const double xmax = (c->sample_type == COBALT_CI8 ? 128.0 : 32768.0) * std::sqrt(2.0);
    const double bound = bmax * sh * xmax * (1.0 + std::ldexp(1.0, -10));
    if (!(bound > 0.0)) return 24;                  // all-zero taps or bandpass: nothing can grow
    const int k = (int)std::floor(std::log2(65504.0 / bound));
    return k > 24 ? 24 : k;
}

int validate(const cobalt_config* c, Sizes* z) {
    if (!c) return fail(COBALT_EINVAL, "cfg is NULL");
    if (c->n_stations < 1) return fail(COBALT_EINVAL, "n_stations must be >= 1 (got %d)", c->n_stations);
    if (c->n_pols != 2) return fail(c->n_pols < 1 ? COBALT_EINVAL : COBALT_EUNSUPPORTED, "n_pols must be 2 (got %d)", c->n_pols);
    if (c->n_subbands < 1) return fail(COBALT_EINVAL, "n_subbands must be >= 1 (got %d)", c->n_subbands);
    if (c->n_channels < 1 || c->n_taps < 1) return fail(COBALT_EINVAL, "n_channels and n_taps must be >= 1");
    if (c->n_channels != 64 && c->n_channels != 256)
        return fail(COBALT_EUNSUPPORTED, "only 64 and 256 channels are built (got %d)", c->n_channels);
    if (c->n_taps != kT) return fail(COBALT_EUNSUPPORTED, "only %d taps are built (got %d)", kT, c->n_taps);
    if (c->sample_type != COBALT_CI8 && c->sample_type != COBALT_CI16 && c->sample_type != COBALT_CF32)
        return fail(COBALT_EINVAL, "unknown sample_type %d", c->sample_type);
    if (c->x_mode != COBALT_X_FP32 && c->x_mode != COBALT_X_FP16_SPLIT && c->x_mode != COBALT_X_INT8)
        return fail(COBALT_EINVAL, "unknown x_mode %d", c->x_mode);
    if (c->samples_per_block < 0 || c->samples_per_block % c->n_channels != 0)
        return fail(COBALT_EINVAL, "samples_per_block (%lld) must be >= 0 and a multiple of n_channels",
                    (long long)c->samples_per_block);
    if (!(c->sample_rate_hz > 0.0) || !std::isfinite(c->sample_rate_hz))
        return fail(COBALT_EINVAL, "sample_rate_hz must be finite and > 0");
    if (c->reserved0 != 0) return fail(COBALT_EINVAL, "reserved0 must be 0");
    if (!c->h_fir) return fail(COBALT_EINVAL, "h_fir is NULL");
    if (!c->h_subband_freq_hz) return fail(COBALT_EINVAL, "h_subband_freq_hz is NULL");
    for (int i = 0; i < kT * c->n_channels; ++i)
        if (!std::isfinite(c->h_fir[i])) return fail(COBALT_EINVAL, "h_fir[%d] is not finite", i);
    if (c->h_bandpass)
        for (int i = 0; i < c->n_channels; ++i)
            if (!std::isfinite(c->h_bandpass[i])) return fail(COBALT_EINVAL, "h_bandpass[%d] is not finite", i);
    for (int i = 0; i < c->n_subbands; ++i)
        if (!std::isfinite(c->h_subband_freq_hz[i])) return fail(COBALT_EINVAL, "h_subband_freq_hz[%d] is not finite", i);

    Sizes s{};
    s.S = c->n_stations; s.P = c->n_pols; s.SB = c->n_subbands; s.C = c->n_channels; s.T = kT;
    s.N = c->samples_per_block; s.n_c = s.N / s.C; s.M = s.S * s.P; s.B = s.S * (s.S + 1) / 2;
    s.pitch = round_up(s.n_c, kPitchAlign);
    s.streams = s.M * s.SB;
    if (s.n_c > (int64_t)1 << 30) return fail(COBALT_EINVAL, "samples_per_block too large");
    if (c->x_mode == COBALT_X_FP32) {
        if (s.M > kMaxFp32Inputs)
            return fail(COBALT_EUNSUPPORTED, "FP32 mode supports up to %d inputs (got %lld)", kMaxFp32Inputs, (long long)s.M);
    } else if (s.M > kMaxMfmaInputs) {
        return fail(COBALT_EUNSUPPORTED, "MFMA modes support up to %d inputs (%d stations); got %lld",
                    kMaxMfmaInputs, kMaxMfmaInputs / 2, (long long)s.M);
    }
    if (c->x_mode == COBALT_X_INT8) {
        if (!(c->requant_gain > 0.f) || !std::isfinite(c->requant_gain))
            return fail(COBALT_EINVAL, "requant_gain must be finite and > 0");
        if (s.n_c * 2 * 127 * 127 >= ((int64_t)1 << 31))
            return fail(COBALT_EOVERFLOW, "INT8 mode: N_c * 2 * 127^2 = %lld overflows int32 (N_c = %lld)",
                        (long long)(s.n_c * 2 * 127 * 127), (long long)s.n_c);
    }
    if (c->x_mode == COBALT_X_FP16_SPLIT) {
        if (c->fp16_prescale_log2 < -24 || c->fp16_prescale_log2 > 24)
            return fail(COBALT_EINVAL, "fp16_prescale_log2 must lie in [-24, 24]");
        const int kmax = fp16_prescale_limit(c);
        if (kmax != INT32_MIN && c->fp16_prescale_log2 > kmax)
            return fail(COBALT_EOVERFLOW,
                        "fp16_prescale_log2 = %d lets full-scale %s samples overflow FP16 with these taps and this "
                        "bandpass; the largest safe value is %d",
                        c->fp16_prescale_log2, c->sample_type == COBALT_CI8 ? "8-bit" : "16-bit", kmax);
    }

    s.sample_bytes = c->sample_type == COBALT_CI8 ? 2 : c->sample_type == COBALT_CI16 ? 4 : 8;
    {
        // kernels address one input stream and one subband's channelised data with 32-bit
        // byte offsets
        const int64_t elem = c->x_mode == COBALT_X_INT8 ? 2 : c->x_mode == COBALT_X_FP16_SPLIT ? 4 : 8;
        const int64_t planes = c->x_mode == COBALT_X_FP16_SPLIT ? 2 : 1;
        if (s.N * s.sample_bytes >= ((int64_t)1 << 31) || s.C * planes * s.M * s.pitch * elem >= ((int64_t)1 << 31))
            return fail(COBALT_EUNSUPPORTED, "block too long: one subband's channelised data must stay below 2 GiB");
    }
    s.input_bytes = s.streams * s.N * s.sample_bytes;
    s.chan_elem_bytes = c->x_mode == COBALT_X_INT8 ? 2 : c->x_mode == COBALT_X_FP16_SPLIT ? 4 : 8;
    s.chan_planes = c->x_mode == COBALT_X_FP16_SPLIT ? 2 : 1;
    s.chan_stride = s.chan_planes * s.M * s.pitch * s.chan_elem_bytes;
    s.chan_bytes = s.SB * s.C * s.chan_stride;
    s.vis_bytes = s.SB * s.C * s.B * 4 * 8;
    s.hist_bytes = s.streams * kHistRows * s.C * s.sample_bytes;
    s.stage_bytes = round_up(s.S * 16 + s.S * 4, 256);         // per ring slot: delays [S][2], offsets [S]
    s.table_bytes = round_up(kT * s.C * 4, 256) + round_up(s.C * 4, 256) + round_up(s.SB * 8, 256) +
                    kRing * s.stage_bytes;
    s.n_words = s.pitch / 32;
    s.cflag_bytes = s.S * s.SB * s.n_words * 4;
    s.rowhist_bytes = s.S * s.SB * 4;
    s.workspace_bytes = round_up(s.chan_bytes, 256) + 2 * round_up(s.hist_bytes, 256) + 2 * round_up(s.rowhist_bytes, 256) +
                        round_up(s.cflag_bytes, 256) + s.table_bytes;
    *z = s;
    return COBALT_OK;
}

}  // namespace

struct cobalt_plan {
    cobalt_config cfg;           // host pointers cleared after create
    Sizes z;
    int device = 0;
    char* d_ws = nullptr;        // one allocation for the whole workspace
    bool owns_ws = true;         // false: the workspace belongs to the caller (service arena)
    void* d_chan = nullptr;
    void* d_hist[2] = {nullptr, nullptr};
    int hist_cur = 0;
    uint32_t* d_rowhist[2] = {nullptr, nullptr};   // lost-sample flags of the rows before the block
    int rowhist_cur = 0;
    bool flag_dirty = false;     // the carried row flags may be nonzero
    uint32_t* d_cflag = nullptr; // flagged channel samples of the current block
    float* d_fir = nullptr;
    float* d_bscale = nullptr;
    double* d_fsb = nullptr;
    char* d_stage[kRing] = {};   // per slot: delays [S][2] float64, coarse offsets [S] int32
    char* h_stage = nullptr;     // pinned [kRing][stage_bytes]
    hipEvent_t ring_ev[kRing] = {};
    bool ring_used[kRing] = {};
    int ring_next = 0;
    hipEvent_t done_ev = nullptr;
    hipStream_t last_stream = nullptr;
    bool has_last = false;
    std::mutex mu;
};

namespace {

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; prev = -1; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int hip_fail(hipError_t e, const char* what) {
    return fail(COBALT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

void free_plan(cobalt_plan* p) {
    if (!p) return;
    for (int i = 0; i < kRing; ++i)
        if (p->ring_ev[i]) (void)hipEventDestroy(p->ring_ev[i]);
    if (p->done_ev) (void)hipEventDestroy(p->done_ev);
    if (p->h_stage) (void)hipHostFree(p->h_stage);
    if (p->d_ws && p->owns_ws) (void)hipFree(p->d_ws);
    delete p;
}

// Order this call after the plan's previous call when it came on another stream.
int begin_call(cobalt_plan* p, hipStream_t st) {
    if (p->has_last && p->last_stream != st) {
        hipError_t e = hipStreamWaitEvent(st, p->done_ev, 0);
        if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    }
    return COBALT_OK;
}

int end_call(cobalt_plan* p, hipStream_t st) {
    hipError_t e = hipEventRecord(p->done_ev, st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    p->last_stream = st;
    p->has_last = true;
    return COBALT_OK;
}

// Copy the caller's delays into a ring slot (pinned host -> device) on stream st.
// Per-call host arrays (residual delays, coarse offsets) go through a pinned ring of kRing
// slots, each guarded by the event of its last copy, so the caller may reuse its arrays at
// once and the copy stays ordered on the call's stream.
int stage_block(cobalt_plan* p, const double* h_delays, const int32_t* h_coarse, int64_t max_offset, hipStream_t st,
                const double** d_delays, const int32_t** d_coarse) {
    const int S = (int)p->z.S;
    for (int i = 0; i < 2 * S; ++i)
        if (!std::isfinite(h_delays[i])) return fail(COBALT_EINVAL, "h_delays[%d] is not finite", i);
    if (h_coarse)
        for (int i = 0; i < S; ++i)
            if (h_coarse[i] < 0 || h_coarse[i] > max_offset)
                return fail(COBALT_EINVAL, "coarse offset of station %d is %d; must lie in 0..%lld", i, h_coarse[i],
                            (long long)max_offset);
    const int slot = p->ring_next;
    p->ring_next = (p->ring_next + 1) % kRing;
    if (p->ring_used[slot]) {
        hipError_t e = hipEventSynchronize(p->ring_ev[slot]);   // the slot's previous copy has run
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    }
    char* h = p->h_stage + (size_t)slot * p->z.stage_bytes;
    std::memcpy(h, h_delays, sizeof(double) * 2 * S);
    const size_t bytes = sizeof(double) * 2 * S + (h_coarse ? sizeof(int32_t) * S : 0);
    if (h_coarse) std::memcpy(h + sizeof(double) * 2 * S, h_coarse, sizeof(int32_t) * S);
    hipError_t e = hipMemcpyAsync(p->d_stage[slot], h, bytes, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(delays)");
    e = hipEventRecord(p->ring_ev[slot], st);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord(delays)");
    p->ring_used[slot] = true;
    *d_delays = (const double*)p->d_stage[slot];
    *d_coarse = h_coarse ? (const int32_t*)(p->d_stage[slot] + sizeof(double) * 2 * S) : nullptr;
    return COBALT_OK;
}

// Flagged channel samples of this block (null when nothing can be flagged: no flags given
// and the carried row flags are known to be clear).
int run_flags(cobalt_plan* p, const uint32_t* d_flags, int64_t row_len, const int32_t* d_coarse, hipStream_t st,
              const uint32_t** cflag) {
    const Sizes& z = p->z;
    *cflag = nullptr;
    if (z.n_c == 0 || (!d_flags && !p->flag_dirty)) return COBALT_OK;
    FlagArgs a{};
    a.flags = d_flags;
    a.flag_words = (row_len + 31) / 32;
    a.coarse = d_coarse;
    a.hist_old = p->d_rowhist[p->rowhist_cur];
    a.hist_new = p->d_rowhist[p->rowhist_cur ^ 1];
    a.cflag = p->d_cflag;
    a.S = (int)z.S;
    a.SB = (int)z.SB;
    a.n_c = (int)z.n_c;
    a.n_words = (int)z.n_words;
    a.C = (int)z.C;
    hipError_t e = launch_chanflags(a, st);
    if (e != hipSuccess) return hip_fail(e, "flag launch");
    p->rowhist_cur ^= 1;
    // the new carried rows are the last T-1 rows of [old rows, block rows]: clear when no
    // flags came in and the block alone spans them
    p->flag_dirty = d_flags != nullptr || (p->flag_dirty && z.n_c < kHistRows);
    *cflag = p->d_cflag;
    return COBALT_OK;
}

FArgs make_fargs(const Sizes& z, const cobalt_config& cfg, const void* d_in, int64_t row_len, const void* hist_old,
                 void* hist_new, const float* fir, const float* bscale, const double* fsb, const double* d_delays,
                 const int32_t* d_coarse, const uint32_t* cflag, void* d_chan) {
    FArgs a{};
    a.in = d_in;
    a.hist_old = hist_old;
    a.hist_new = hist_new;
    a.out = d_chan;
    a.fir = fir;
    a.bscale = bscale;
    a.f_sb = fsb;
    a.delays = d_delays;
    a.coarse = d_coarse;
    a.cflag = cflag;
    a.N = z.N;
    a.row_len = row_len;
    a.n_words = (int)z.n_words;
    a.S = (int)z.S;
    a.SB = (int)z.SB;
    a.M = (int)z.M;
    a.n_c = (int)z.n_c;
    a.pitch = (int)z.pitch;
    a.n_chunks = (int)((z.pitch + kFChunk - 1) / kFChunk);
    a.n_kb = (int)(z.pitch / kKBlock);
    a.df = cfg.sample_rate_hz / (double)z.C;
    a.C = (int)z.C;
    return a;
}

XArgs make_xargs(const Sizes& z, const cobalt_config& cfg, const void* d_chan, void* d_vis) {
    XArgs a{};
    a.chan = d_chan;
    a.vis = d_vis;
    a.chan_stride = z.chan_stride;
    a.M = (int)z.M;
    a.S = (int)z.S;
    a.n_c = (int)z.n_c;
    a.pitch = (int)z.pitch;
    a.n_chan = (int)(z.SB * z.C);
    a.n_blocks8 = (int)((z.M + 7) / 8);
    a.n_kb = (int)(z.pitch / kKBlock);
    a.out_scale = std::ldexp(1.0f, -2 * cfg.fp16_prescale_log2);
    return a;
}

int launch_x(const cobalt_config& cfg, const XArgs& a, hipStream_t st) {
    hipError_t e = cfg.x_mode == COBALT_X_FP32 ? launch_xstage_fp32(a, st) : launch_xstage_mfma(cfg.x_mode, a, st);
    if (e != hipSuccess) return hip_fail(e, "X-stage launch");
    return COBALT_OK;
}

int run_fstage(cobalt_plan* p, const void* d_in, int64_t row_len, const double* d_delays, const int32_t* d_coarse,
               const uint32_t* cflag, void* d_chan, hipStream_t st) {
    const Sizes& z = p->z;
    if (z.n_c == 0) return COBALT_OK;       // empty block: nothing to filter, history unchanged
    const FArgs a = make_fargs(z, p->cfg, d_in, row_len, p->d_hist[p->hist_cur], p->d_hist[p->hist_cur ^ 1], p->d_fir,
                               p->d_bscale, p->d_fsb, d_delays, d_coarse, cflag, d_chan);
    hipError_t e = launch_fstage(p->cfg.sample_type, p->cfg.x_mode, a, (int)z.streams, st);
    if (e != hipSuccess) return hip_fail(e, "F-stage launch");
    p->hist_cur ^= 1;
    return COBALT_OK;
}

int run_xstage(cobalt_plan* p, const void* d_chan, void* d_vis, hipStream_t st) {
    return launch_x(p->cfg, make_xargs(p->z, p->cfg, d_chan, d_vis), st);
}

struct CallLock {
    std::unique_lock<std::mutex> lk;
    explicit CallLock(cobalt_plan* p) : lk(p->mu, std::try_to_lock) {}
    bool owns() const { return lk.owns_lock(); }
};

}  // namespace

extern "C" {

const char* cobalt_last_error(void) { return g_last_error.c_str(); }

int cobalt_estimate_bytes(const cobalt_config* cfg, size_t* device_bytes) {
    g_last_error.clear();
    if (!device_bytes) return fail(COBALT_EINVAL, "device_bytes is NULL");
    Sizes z;
    int rc = validate(cfg, &z);
    if (rc != COBALT_OK) return rc;
    *device_bytes = (size_t)z.workspace_bytes;
    return COBALT_OK;
}

int cobalt_fp16_prescale_max(const cobalt_config* cfg, int32_t* k_max) {
    g_last_error.clear();
    if (!k_max) return fail(COBALT_EINVAL, "k_max is NULL");
    if (!cfg) return fail(COBALT_EINVAL, "cfg is NULL");
    cobalt_config c = *cfg;                  // the rest of the setting must be valid
    c.x_mode = COBALT_X_FP16_SPLIT;
    c.fp16_prescale_log2 = -24;
    Sizes z;
    int rc = validate(&c, &z);
    if (rc != COBALT_OK) return rc;
    const int k = fp16_prescale_limit(&c);
    if (k == INT32_MIN) return fail(COBALT_EINVAL, "float samples have no fixed bound; the caller chooses the prescale");
    *k_max = k;
    return COBALT_OK;
}

}  // extern "C"

// Plan creation with the workspace either allocated here or given by the caller (the
// streaming service carves observation workspaces out of one device arena).  The tables
// and the zeroed history are uploaded on a private stream that is synchronised before
// return, so creating a plan does not wait for work other plans have queued on the device.
int cobalt::plan_create_impl(const cobalt_config* cfg, void* d_workspace, cobalt_plan** out) {
    g_last_error.clear();
    if (!out) return fail(COBALT_EINVAL, "out is NULL");
    *out = nullptr;
    Sizes z;
    int rc = validate(cfg, &z);
    if (rc != COBALT_OK) return rc;
    if (d_workspace && (uintptr_t)d_workspace % 256) return fail(COBALT_EINVAL, "workspace must be 256-byte aligned");

    cobalt_plan* p = new (std::nothrow) cobalt_plan();
    if (!p) return fail(COBALT_ENOMEM, "host allocation failed");
    p->cfg = *cfg;
    p->cfg.h_fir = nullptr;
    p->cfg.h_bandpass = nullptr;
    p->cfg.h_subband_freq_hz = nullptr;
    p->z = z;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) { free_plan(p); return hip_fail(e, "hipGetDevice"); }

    if (d_workspace) {
        p->d_ws = (char*)d_workspace;
        p->owns_ws = false;
    } else {
        e = hipMalloc((void**)&p->d_ws, (size_t)z.workspace_bytes);
        if (e != hipSuccess) {
            p->d_ws = nullptr;
            free_plan(p);
            (void)hipGetLastError();
            return fail(COBALT_ENOMEM, "hipMalloc(%lld bytes) failed: %s", (long long)z.workspace_bytes, hipGetErrorString(e));
        }
    }
    char* q = p->d_ws;
    p->d_chan = q;                q += round_up(z.chan_bytes, 256);
    p->d_hist[0] = q;             q += round_up(z.hist_bytes, 256);
    p->d_hist[1] = q;             q += round_up(z.hist_bytes, 256);
    p->d_rowhist[0] = (uint32_t*)q; q += round_up(z.rowhist_bytes, 256);
    p->d_rowhist[1] = (uint32_t*)q; q += round_up(z.rowhist_bytes, 256);
    p->d_cflag = (uint32_t*)q;    q += round_up(z.cflag_bytes, 256);
    p->d_fir = (float*)q;         q += round_up(kT * z.C * 4, 256);
    p->d_bscale = (float*)q;      q += round_up(z.C * 4, 256);
    p->d_fsb = (double*)q;        q += round_up(z.SB * 8, 256);
    for (int i = 0; i < kRing; ++i) { p->d_stage[i] = q; q += z.stage_bytes; }

    e = hipHostMalloc((void**)&p->h_stage, (size_t)z.stage_bytes * kRing, hipHostMallocDefault);
    if (e != hipSuccess) { free_plan(p); (void)hipGetLastError(); return fail(COBALT_ENOMEM, "hipHostMalloc failed"); }
    for (int i = 0; i < kRing; ++i) {
        e = hipEventCreateWithFlags(&p->ring_ev[i], hipEventDisableTiming);
        if (e != hipSuccess) { free_plan(p); return hip_fail(e, "hipEventCreate"); }
    }
    e = hipEventCreateWithFlags(&p->done_ev, hipEventDisableTiming);
    if (e != hipSuccess) { free_plan(p); return hip_fail(e, "hipEventCreate"); }

    // tables: FIR, bandpass x mode scale (2^k, requant gain, or 1), subband frequencies
    float bscale[256];
    const double mode_scale = cfg->x_mode == COBALT_X_FP16_SPLIT ? std::ldexp(1.0, cfg->fp16_prescale_log2)
                              : cfg->x_mode == COBALT_X_INT8   ? (double)cfg->requant_gain
                                                               : 1.0;
    for (int c = 0; c < z.C; ++c) bscale[c] = (float)((cfg->h_bandpass ? (double)cfg->h_bandpass[c] : 1.0) * mode_scale);
    hipStream_t init = nullptr;
    e = hipStreamCreateWithFlags(&init, hipStreamNonBlocking);
    if (e != hipSuccess) { free_plan(p); return hip_fail(e, "hipStreamCreate"); }
    e = hipMemcpyAsync(p->d_fir, cfg->h_fir, sizeof(float) * kT * z.C, hipMemcpyHostToDevice, init);
    if (e == hipSuccess) e = hipMemcpyAsync(p->d_bscale, bscale, sizeof(float) * z.C, hipMemcpyHostToDevice, init);
    if (e == hipSuccess) e = hipMemcpyAsync(p->d_fsb, cfg->h_subband_freq_hz, sizeof(double) * z.SB, hipMemcpyHostToDevice, init);
    // FIR history starts at zero (no samples before the first block), its rows unflagged
    if (e == hipSuccess)
        e = launch_zero_fill(p->d_hist[0], round_up(z.hist_bytes, 256) * 2 + round_up(z.rowhist_bytes, 256) * 2, init);
    const hipError_t es = hipStreamSynchronize(init);   // the host tables may be freed after return
    if (e == hipSuccess) e = es;
    (void)hipStreamDestroy(init);
    if (e != hipSuccess) { free_plan(p); return hip_fail(e, "table upload / history init"); }
    *out = p;
    return COBALT_OK;
}

extern "C" {

int cobalt_plan_create(const cobalt_config* cfg, cobalt_plan** out) { return plan_create_impl(cfg, nullptr, out); }

int cobalt_plan_query(const cobalt_plan* p, cobalt_plan_info* info) {
    g_last_error.clear();
    if (!p || !info) return fail(COBALT_EINVAL, "plan or info is NULL");
    const Sizes& z = p->z;
    info->n_channel_samples = z.n_c;
    info->chan_pitch = z.pitch;
    info->n_baselines = z.B;
    info->input_bytes = z.input_bytes;
    info->chan_bytes = z.chan_bytes;
    info->vis_bytes = z.vis_bytes;
    info->workspace_bytes = z.workspace_bytes;
    info->useful_cmacs = z.B * 4 * z.SB * z.C * z.n_c;
    return COBALT_OK;
}

static int do_fx(cobalt_plan* p, const void* d_in, const double* h_delays, const cobalt_block_ext* ext, void* d_chan,
                 void* d_vis, void* stream) {
    g_last_error.clear();
    if (!p) return fail(COBALT_EINVAL, "plan is NULL");
    if ((!d_in && p->z.input_bytes > 0) || !h_delays) return fail(COBALT_EINVAL, "d_in or h_delays is NULL");
    if (!d_chan && !d_vis) return fail(COBALT_EINVAL, "output pointer is NULL");
    if (((uintptr_t)d_in | (uintptr_t)d_chan | (uintptr_t)d_vis) % 16)
        return fail(COBALT_EINVAL, "device pointers must be 16-byte aligned");
    const Sizes& z = p->z;
    int64_t row_len = z.N;
    const int32_t* h_coarse = nullptr;
    const uint32_t* d_flags = nullptr;
    int32_t* d_weights = nullptr;
    if (ext) {
        if (ext->row_samples != 0) {
            if (ext->row_samples < z.N) return fail(COBALT_EINVAL, "row_samples (%lld) is below N (%lld)",
                                                    (long long)ext->row_samples, (long long)z.N);
            if (ext->row_samples > ((int64_t)1 << 40)) return fail(COBALT_EINVAL, "row_samples too large");
            row_len = ext->row_samples;
        }
        h_coarse = ext->h_coarse_offset;
        d_flags = ext->d_flags;
        d_weights = ext->d_weights;
        if (((uintptr_t)d_flags | (uintptr_t)d_weights) % 4)
            return fail(COBALT_EINVAL, "d_flags and d_weights must be 4-byte aligned");
    }
    CallLock lock(p);
    if (!lock.owns()) return fail(COBALT_EBUSY, "plan is in use by another host thread");
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(COBALT_EDEVICE, "cannot select the plan's device");
    hipStream_t st = (hipStream_t)stream;
    int rc = begin_call(p, st);
    if (rc) return rc;
    const double* d_delays = nullptr;
    const int32_t* d_coarse = nullptr;
    rc = stage_block(p, h_delays, h_coarse, row_len - z.N, st, &d_delays, &d_coarse);
    if (rc) return rc;
    const uint32_t* cflag = nullptr;
    rc = run_flags(p, d_flags, row_len, d_coarse, st, &cflag);
    if (rc) return rc;
    void* chan = d_chan ? d_chan : p->d_chan;
    rc = run_fstage(p, d_in, row_len, d_delays, d_coarse, cflag, chan, st);
    if (rc) return rc;
    if (d_weights) {
        hipError_t e = launch_weights(cflag, d_weights, (int)z.S, (int)z.SB, (int)z.n_c, (int)z.n_words, st);
        if (e != hipSuccess) return hip_fail(e, "weights launch");
    }
    if (d_vis) {
        rc = run_xstage(p, chan, d_vis, st);
        if (rc) return rc;
    }
    return end_call(p, st);
}

int cobalt_correlate(cobalt_plan* p, const void* d_in, const double* h_delays, void* d_vis, void* stream) {
    if (!d_vis) { g_last_error = "d_vis is NULL"; return COBALT_EINVAL; }
    return do_fx(p, d_in, h_delays, nullptr, nullptr, d_vis, stream);
}

int cobalt_channelize(cobalt_plan* p, const void* d_in, const double* h_delays, void* d_chan, void* stream) {
    if (!d_chan) { g_last_error = "d_chan is NULL"; return COBALT_EINVAL; }
    return do_fx(p, d_in, h_delays, nullptr, d_chan, nullptr, stream);
}

int cobalt_correlate_ex(cobalt_plan* p, const void* d_in, const double* h_delays, const cobalt_block_ext* ext, void* d_vis,
                        void* stream) {
    if (!d_vis) { g_last_error = "d_vis is NULL"; return COBALT_EINVAL; }
    return do_fx(p, d_in, h_delays, ext, nullptr, d_vis, stream);
}

int cobalt_channelize_ex(cobalt_plan* p, const void* d_in, const double* h_delays, const cobalt_block_ext* ext, void* d_chan,
                         void* stream) {
    if (!d_chan) { g_last_error = "d_chan is NULL"; return COBALT_EINVAL; }
    return do_fx(p, d_in, h_delays, ext, d_chan, nullptr, stream);
}

// ---- beamformer ----
static int check_beam(const cobalt_plan* p, const cobalt_beam_params* bp, const void* coh, const void* volt, const void* inc) {
    const Sizes& z = p->z;
    if (!bp) return fail(COBALT_EINVAL, "beam parameters are NULL");
    if (p->cfg.x_mode != COBALT_X_FP16_SPLIT) return fail(COBALT_EUNSUPPORTED, "the beamformer needs an FP16-split plan");
    if (z.S > 56) return fail(COBALT_EUNSUPPORTED, "the beamformer supports up to 56 stations (got %lld)", (long long)z.S);
    if (bp->n_beams < 1) return fail(COBALT_EINVAL, "n_beams must be >= 1 (got %d)", bp->n_beams);
    if (bp->n_stokes != 1 && bp->n_stokes != 4) return fail(COBALT_EINVAL, "n_stokes must be 1 or 4 (got %d)", bp->n_stokes);
    if (bp->voltage_stride != 0 && (bp->voltage_stride < bp->n_beams || bp->voltage_stride > 65536))
        return fail(COBALT_EINVAL, "voltage_stride must be 0 or in [n_beams, 65536] (got %d)", bp->voltage_stride);
    const int ni = bp->n_int;
    const bool pow2 = ni >= 1 && ni <= 32 && (ni & (ni - 1)) == 0;
    if (!(pow2 || (ni > 32 && ni % 32 == 0))) return fail(COBALT_EINVAL, "n_int must be a power of two <= 32 or a multiple of 32 (got %d)", ni);
    if (z.n_c % ni != 0) return fail(COBALT_EINVAL, "n_int (%d) must divide N_c (%lld)", ni, (long long)z.n_c);
    if (!bp->d_beam_dtau || (uintptr_t)bp->d_beam_dtau % 8) return fail(COBALT_EINVAL, "d_beam_dtau is NULL or misaligned");
    if (!coh && !volt && !inc) return fail(COBALT_EINVAL, "no output requested");
    if (((uintptr_t)coh | (uintptr_t)volt | (uintptr_t)inc) % 16) return fail(COBALT_EINVAL, "outputs must be 16-byte aligned");
    return COBALT_OK;
}

static int run_beam(cobalt_plan* p, const void* chan, const cobalt_beam_params* bp, void* coh, void* volt, void* inc,
                    hipStream_t st) {
    const Sizes& z = p->z;
    BeamArgs a{};
    a.chan = chan;
    a.chan_stride = z.chan_stride;
    a.f_sb = p->d_fsb;
    a.dtau = bp->d_beam_dtau;
    a.coherent = coh;
    a.voltages = volt;
    a.incoherent = inc;
    a.df = p->cfg.sample_rate_hz / (double)z.C;
    a.C = (int)z.C;
    a.S = (int)z.S;
    a.NB = bp->n_beams;
    a.vstride = bp->voltage_stride ? bp->voltage_stride : bp->n_beams;
    a.n_c = (int)z.n_c;
    a.n_kb = (int)(z.pitch / kKBlock);
    a.n_chan = (int)(z.SB * z.C);
    a.n_int = bp->n_int;
    a.n_stokes = bp->n_stokes;
    a.vscale = std::ldexp(1.0f, -p->cfg.fp16_prescale_log2);
    if (z.n_c == 0) return COBALT_OK;
    hipError_t e = launch_beamformer(a, st);
    if (e != hipSuccess) return hip_fail(e, "beamformer launch");
    return COBALT_OK;
}

int cobalt_beamform(cobalt_plan* p, const void* d_in, const double* h_delays, const cobalt_beam_params* bp, void* d_coherent,
                    void* d_voltages, void* d_incoherent, void* stream) {
    g_last_error.clear();
    if (!p) return fail(COBALT_EINVAL, "plan is NULL");
    int rc = check_beam(p, bp, d_coherent, d_voltages, d_incoherent);
    if (rc) return rc;
    if ((!d_in && p->z.input_bytes > 0) || !h_delays) return fail(COBALT_EINVAL, "d_in or h_delays is NULL");
    if ((uintptr_t)d_in % 16) return fail(COBALT_EINVAL, "device pointers must be 16-byte aligned");
    CallLock lock(p);
    if (!lock.owns()) return fail(COBALT_EBUSY, "plan is in use by another host thread");
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(COBALT_EDEVICE, "cannot select the plan's device");
    hipStream_t st = (hipStream_t)stream;
    rc = begin_call(p, st);
    if (rc) return rc;
    const double* d_delays = nullptr;
    const int32_t* d_coarse = nullptr;
    rc = stage_block(p, h_delays, nullptr, 0, st, &d_delays, &d_coarse);
    if (rc) return rc;
    const uint32_t* cflag = nullptr;
    rc = run_flags(p, nullptr, p->z.N, nullptr, st, &cflag);
    if (rc) return rc;
    rc = run_fstage(p, d_in, p->z.N, d_delays, nullptr, cflag, p->d_chan, st);
    if (rc) return rc;
    rc = run_beam(p, p->d_chan, bp, d_coherent, d_voltages, d_incoherent, st);
    if (rc) return rc;
    return end_call(p, st);
}

int cobalt_beamform_channelized(cobalt_plan* p, const void* d_chan, const cobalt_beam_params* bp, void* d_coherent,
                                void* d_voltages, void* d_incoherent, void* stream) {
    g_last_error.clear();
    if (!p) return fail(COBALT_EINVAL, "plan is NULL");
    int rc = check_beam(p, bp, d_coherent, d_voltages, d_incoherent);
    if (rc) return rc;
    if ((!d_chan && p->z.chan_bytes > 0) || (uintptr_t)d_chan % 16) return fail(COBALT_EINVAL, "d_chan is NULL or misaligned");
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(COBALT_EDEVICE, "cannot select the plan's device");
    return run_beam(p, d_chan, bp, d_coherent, d_voltages, d_incoherent, (hipStream_t)stream);
}

int cobalt_beam_transform(cobalt_plan* p, const void* d_voltages, const cobalt_transform_params* tp,
                          void* d_out_voltages, void* d_out_stokes, void* stream) {
    g_last_error.clear();
    if (!p) return fail(COBALT_EINVAL, "plan is NULL");
    if (!tp) return fail(COBALT_EINVAL, "transform parameters are NULL");
    const Sizes& z = p->z;
    if (z.C != 256) return fail(COBALT_EUNSUPPORTED, "the transform takes 256-channel voltages (plan has %lld)", (long long)z.C);
    if (tp->n_beams < 1) return fail(COBALT_EINVAL, "n_beams must be >= 1 (got %d)", tp->n_beams);
    const int co = tp->c_out;
    if (co != 1 && co != 2 && co != 4 && co != 8 && co != 16)
        return fail(COBALT_EUNSUPPORTED, "c_out must be 1, 2, 4, 8 or 16 (got %d)", co);
    if (tp->voltage_stride != 0 && (tp->voltage_stride < tp->n_beams || tp->voltage_stride > 65536))
        return fail(COBALT_EINVAL, "voltage_stride must be 0 or in [n_beams, 65536] (got %d)", tp->voltage_stride);
    const int64_t nbs = tp->voltage_stride ? tp->voltage_stride : tp->n_beams;
    if (!d_out_voltages && !d_out_stokes) return fail(COBALT_EINVAL, "no output requested");
    if (d_out_stokes) {
        if (tp->n_stokes != 1 && tp->n_stokes != 4) return fail(COBALT_EINVAL, "n_stokes must be 1 or 4 (got %d)", tp->n_stokes);
        const int per_row = 256 / co, ni = tp->n_int;
        if (ni < 1 || (ni & (ni - 1)) != 0 || ni > per_row)
            return fail(COBALT_EINVAL, "n_int must be a power of two up to %d (got %d)", per_row, ni);
    }
    if ((!d_voltages && z.n_c > 0) || ((uintptr_t)d_voltages | (uintptr_t)d_out_voltages | (uintptr_t)d_out_stokes) % 16)
        return fail(COBALT_EINVAL, "device pointers must be non-NULL and 16-byte aligned");
    if ((int64_t)z.SB * z.n_c >= ((int64_t)1 << 31))
        return fail(COBALT_EUNSUPPORTED, "too many subbands x channel samples for one launch");
    // the kernel addresses one subband's voltages with 32-bit byte offsets
    if ((int64_t)256 * z.n_c * 2 * nbs * 8 >= ((int64_t)1 << 32))
        return fail(COBALT_EUNSUPPORTED, "one subband's voltages must stay below 4 GiB (channel samples x beam stride = "
                    "%lld, at most %lld)", (long long)(z.n_c * nbs), (long long)(((int64_t)1 << 32) / 4096) - 1);
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(COBALT_EDEVICE, "cannot select the plan's device");
    TfArgs a{};
    a.vin = d_voltages;
    a.vout = d_out_voltages;
    a.sout = d_out_stokes;
    a.SB = (int)z.SB;
    a.n_c = (int)z.n_c;
    a.NB = tp->n_beams;
    a.vstride = (int32_t)nbs;
    a.n_bg = (tp->n_beams + 15) / 16;
    a.c_out = co;
    a.n_stokes = d_out_stokes ? tp->n_stokes : 0;
    a.n_int = d_out_stokes ? tp->n_int : 1;
    hipError_t e = launch_beam_transform(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "transform launch");
    return COBALT_OK;
}

// Stateless with respect to the plan (reads only its immutable sizes): ordered by the
// caller's stream alone, so it can overlap the plan's F-stage calls on another stream.
int cobalt_correlate_channelized(cobalt_plan* p, const void* d_chan, void* d_vis, void* stream) {
    g_last_error.clear();
    if (!p) return fail(COBALT_EINVAL, "plan is NULL");
    if ((!d_chan && p->z.chan_bytes > 0) || !d_vis) return fail(COBALT_EINVAL, "d_chan or d_vis is NULL");
    if (((uintptr_t)d_chan | (uintptr_t)d_vis) % 16) return fail(COBALT_EINVAL, "device pointers must be 16-byte aligned");
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(COBALT_EDEVICE, "cannot select the plan's device");
    return run_xstage(p, d_chan, d_vis, (hipStream_t)stream);
}

int cobalt_reset_history(cobalt_plan* p, void* stream) {
    g_last_error.clear();
    if (!p) return fail(COBALT_EINVAL, "plan is NULL");
    CallLock lock(p);
    if (!lock.owns()) return fail(COBALT_EBUSY, "plan is in use by another host thread");
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(COBALT_EDEVICE, "cannot select the plan's device");
    hipStream_t st = (hipStream_t)stream;
    int rc = begin_call(p, st);
    if (rc) return rc;
    hipError_t e = launch_zero_fill(p->d_hist[p->hist_cur], round_up(p->z.hist_bytes, 256), st);
    if (e == hipSuccess) e = launch_zero_fill(p->d_rowhist[p->rowhist_cur], round_up(p->z.rowhist_bytes, 256), st);
    if (e != hipSuccess) return hip_fail(e, "history reset");
    p->flag_dirty = false;
    return end_call(p, st);
}

// Stateless like cobalt_correlate_channelized: ordered by the caller's stream alone.
static int gains_call(cobalt_plan* p, const void* a0, const void* a1, const void* a2, void* out, void* stream, bool adjoint) {
    g_last_error.clear();
    if (!p) return fail(COBALT_EINVAL, "plan is NULL");
    if (p->cfg.x_mode == COBALT_X_INT8) return fail(COBALT_EUNSUPPORTED, "gains need float visibilities (FP32 or FP16-split mode)");
    if (!a0 || !a1 || (adjoint && !a2) || !out) return fail(COBALT_EINVAL, "NULL device pointer");
    if (((uintptr_t)a0 | (uintptr_t)a1 | (uintptr_t)a2 | (uintptr_t)out) % 16)
        return fail(COBALT_EINVAL, "device pointers must be 16-byte aligned");
    DeviceGuard dg(p->device);
    if (!dg.ok) return fail(COBALT_EDEVICE, "cannot select the plan's device");
    hipStream_t st = (hipStream_t)stream;
    const int n_chan = (int)(p->z.SB * p->z.C), S = (int)p->z.S;
    hipError_t e = adjoint ? launch_apply_gains_adjoint(a0, a1, a2, out, n_chan, S, st)
                           : launch_apply_gains(a0, a1, out, n_chan, S, st);
    if (e != hipSuccess) return hip_fail(e, adjoint ? "gain adjoint launch" : "gain launch");
    return COBALT_OK;
}

int cobalt_apply_gains(cobalt_plan* p, const void* d_vis0, const void* d_gains, void* d_vis, void* stream) {
    return gains_call(p, d_vis0, d_gains, nullptr, d_vis, stream, false);
}

int cobalt_apply_gains_adjoint(cobalt_plan* p, const void* d_vis0, const void* d_gains, const void* d_grad_vis,
                               void* d_grad_gains, void* stream) {
    return gains_call(p, d_vis0, d_gains, d_grad_vis, d_grad_gains, stream, true);
}

int cobalt_device_copy(void* d_dst, const void* d_src, size_t bytes, void* stream) {
    g_last_error.clear();
    if ((!d_dst || !d_src) && bytes > 0) return fail(COBALT_EINVAL, "NULL device pointer");
    if (((uintptr_t)d_dst | (uintptr_t)d_src | bytes) % 16) return fail(COBALT_EINVAL, "pointers and size must be multiples of 16 bytes");
    hipError_t e = launch_device_copy(d_dst, d_src, (int64_t)bytes, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "copy launch");
    return COBALT_OK;
}

int cobalt_device_fanout(void* d_dst0, void* d_dst1, const void* d_src, size_t bytes, void* stream) {
    g_last_error.clear();
    if ((!d_dst0 || !d_dst1 || !d_src) && bytes > 0) return fail(COBALT_EINVAL, "NULL device pointer");
    if (((uintptr_t)d_dst0 | (uintptr_t)d_dst1 | (uintptr_t)d_src | bytes) % 16)
        return fail(COBALT_EINVAL, "pointers and size must be multiples of 16 bytes");
    hipError_t e = launch_device_fanout(d_dst0, d_dst1, d_src, (int64_t)bytes, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "fan-out launch");
    return COBALT_OK;
}

int cobalt_mfma_probe(int32_t x_mode, int64_t iterations, int32_t workgroups, float* d_sink, void* stream) {
    g_last_error.clear();
    if (x_mode != COBALT_X_FP16_SPLIT && x_mode != COBALT_X_INT8)
        return fail(COBALT_EINVAL, "x_mode must be FP16-split or int8 (got %d)", x_mode);
    if (iterations < 1 || iterations > ((int64_t)1 << 19)) return fail(COBALT_EINVAL, "iterations must be 1 .. 2^19");
    if (workgroups < 1 || workgroups > (1 << 20)) return fail(COBALT_EINVAL, "workgroups must be 1 .. 2^20");
    if (!d_sink) return fail(COBALT_EINVAL, "NULL sink");
    if ((uintptr_t)d_sink % 4) return fail(COBALT_EINVAL, "sink must be 4-byte aligned");
    hipError_t e = launch_mfma_probe(x_mode, iterations, workgroups, d_sink, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "probe launch");
    return COBALT_OK;
}

}  // extern "C"

// ---- the entry point that allocates nothing --------------------------------------------
// Scratch for cobalt_correlate_noalloc: the channelised block between its F and X stages,
// the zero or discarded FIR history when the caller passes none, and the per-call tables.
// Every GPU the library runs on holds one copy for the life of the process.
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
char* g_scratch_ptr[64] = {};      // device address of `scratch` per device, looked up once

// The device address of this device's `scratch` (the host-side symbol is only a stand-in).
int scratch_base(char** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= 64) return fail(COBALT_EDEVICE, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = (char*)ptr;
    }
    *out = g_scratch_ptr[dev];
    return COBALT_OK;
}

}  // namespace

extern "C" {

int cobalt_correlate_noalloc(const cobalt_config* cfg, const void* d_in, const double* h_delays, const void* d_hist_in,
                             void* d_hist_out, void* d_vis, void* stream) {
    g_last_error.clear();
    Sizes z;
    int rc = validate(cfg, &z);
    if (rc != COBALT_OK) return rc;
    if (z.N == 0) return fail(COBALT_EINVAL, "samples_per_block must be > 0 for this entry point");
    if (!d_in || !h_delays || !d_vis) return fail(COBALT_EINVAL, "d_in, h_delays or d_vis is NULL");
    if (((uintptr_t)d_in | (uintptr_t)d_vis | (uintptr_t)d_hist_in | (uintptr_t)d_hist_out) % 16)
        return fail(COBALT_EINVAL, "device pointers must be 16-byte aligned");
    if (d_hist_in && d_hist_in == d_hist_out)
        return fail(COBALT_EINVAL, "d_hist_in and d_hist_out must differ (the F stage reads one while writing the other)");
    for (int i = 0; i < 2 * z.S; ++i)
        if (!std::isfinite(h_delays[i])) return fail(COBALT_EINVAL, "h_delays[%d] is not finite", i);
    // scratch layout: channelised block | zero history | discarded history | FIR | bandpass x scale |
    // subband frequencies | delays
    const int64_t hist = round_up(z.hist_bytes, 256);
    const int64_t o_chan = 0;
    const int64_t o_hzero = o_chan + round_up(z.chan_bytes, 256);
    const int64_t o_hdrop = o_hzero + (d_hist_in ? 0 : hist);
    const int64_t o_fir = o_hdrop + (d_hist_out ? 0 : hist);
    const int64_t o_bsc = o_fir + round_up(kT * z.C * 4, 256);
    const int64_t o_fsb = o_bsc + round_up(z.C * 4, 256);
    const int64_t o_del = o_fsb + round_up(z.SB * 8, 256);
    const int64_t total = o_del + round_up(z.S * 16, 256);
    if (total > (int64_t)kScratchBytes)
        return fail(COBALT_EUNSUPPORTED,
                    "this setting needs %lld bytes of scratch; the no-allocation entry point has %zu (use a plan)",
                    (long long)total, kScratchBytes);
    char* base = nullptr;
    rc = scratch_base(&base);
    if (rc != COBALT_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    float bscale[256];
    const double mode_scale = cfg->x_mode == COBALT_X_FP16_SPLIT ? std::ldexp(1.0, cfg->fp16_prescale_log2)
                              : cfg->x_mode == COBALT_X_INT8   ? (double)cfg->requant_gain
                                                               : 1.0;
    for (int c = 0; c < z.C; ++c) bscale[c] = (float)((cfg->h_bandpass ? (double)cfg->h_bandpass[c] : 1.0) * mode_scale);
    // host -> scratch copies from pageable memory return once the source has been read
    hipError_t e = hipMemcpyAsync(base + o_fir, cfg->h_fir, sizeof(float) * kT * z.C, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(base + o_bsc, bscale, sizeof(float) * z.C, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(base + o_fsb, cfg->h_subband_freq_hz, sizeof(double) * z.SB, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(base + o_del, h_delays, sizeof(double) * 2 * z.S, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "table upload");
    if (!d_hist_in) {
        e = launch_zero_fill(base + o_hzero, hist, st);      // a fill kernel, no memset node
        if (e != hipSuccess) return hip_fail(e, "history fill");
    }
    const FArgs a = make_fargs(z, *cfg, d_in, z.N, d_hist_in ? d_hist_in : base + o_hzero,
                               d_hist_out ? d_hist_out : base + o_hdrop, (const float*)(base + o_fir),
                               (const float*)(base + o_bsc), (const double*)(base + o_fsb),
                               (const double*)(base + o_del), nullptr, nullptr, base + o_chan);
    e = launch_fstage(cfg->sample_type, cfg->x_mode, a, (int)z.streams, st);
    if (e != hipSuccess) return hip_fail(e, "F-stage launch");
    return launch_x(*cfg, make_xargs(z, *cfg, base + o_chan, d_vis), st);
}

int cobalt_plan_destroy(cobalt_plan* p) {
    g_last_error.clear();
    if (!p) return COBALT_OK;
    int rc = COBALT_OK;
    {
        DeviceGuard dg(p->device);
        if (p->has_last) {
            hipError_t e = hipEventSynchronize(p->done_ev);
            if (e != hipSuccess) rc = hip_fail(e, "hipEventSynchronize(destroy)");
        }
        free_plan(p);
    }
    return rc;
}

}  // extern "C"

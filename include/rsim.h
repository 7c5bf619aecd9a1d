/*
 * rsim.h -- C ABI of the MI355X room-simulator hot path (librsim.so).
 *
 * The library implements, with hand-written HIP kernels for gfx950:
 *   - the RIR tail cut-off of Sec. 2.3, eqs. (7)-(9);
 *   - overlap-add FFT filtering of Sec. 2.2 (eq. (6) and the text around it),
 *     which reproduces the linear convolution h_ij * x_i of eq. (2);
 *   - the mixing model of eq. (2), y_j = sum_i alpha_ij (h_ij * x_i);
 *   - the adjoint of eq. (2) with respect to x, h and alpha.
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers unless marked (host).  The caller
 *     owns every buffer; the library never frees or keeps caller memory.
 *   - Calls that take a hipStream_t are asynchronous on that stream.  Their
 *     return code reports only synchronous host-side validation; problems the
 *     host cannot see (bad offsets inside device descriptor arrays, non-finite
 *     RIR samples) set bits of a per-device status word read with
 *     rsim_device_status().  Such items are skipped, never read out of bounds.
 *   - No call allocates device memory after rsim_init(): scratch space comes
 *     from the `ws` argument, sized by the matching *_workspace_bytes() call.
 *   - No call aborts or throws across the ABI.
 *   - All sample data is float32.  Lengths and counts are int32, offsets int64
 *     (in elements, not bytes).
 */
#ifndef RSIM_H
#define RSIM_H

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RSIM_OK = 0,
  RSIM_EINVAL = 1,       /* bad argument (null pointer, negative size, eta < 0 or NaN, ...) */
  RSIM_EWORKSPACE = 2,   /* ws is null or smaller than the *_workspace_bytes() value */
  RSIM_EUNSUPPORTED = 3, /* FFT size not a power of two in [512, 32768], or hop/RIR do not fit */
  RSIM_EDEVICE = 4,      /* a HIP runtime call failed (launch, graph, copy) */
  RSIM_ENOTINIT = 5      /* first use on this device happened during stream capture */
} rsim_status;

/* Bits of the device status word (rsim_device_status). */
#define RSIM_DEV_NONFINITE 0x1 /* a RIR had a non-finite sample or h^2 overflowed: kept uncut */
#define RSIM_DEV_BADDESC 0x2   /* a descriptor entry was out of range: that item was skipped */
#define RSIM_DEV_BADPLAN 0x4   /* a requested FFT size / hop did not fit an utterance: skipped */

/*
 * Batch descriptor.  Scalars are host values; pointers are device arrays.
 * U = n_utt utterances, J = n_mic microphones, S = max_src source slots per
 * utterance (source 0 is the target).  RIR (u, i, j) has index
 * r = (u*S + i)*J + j; source (u, i) has index u*S + i.
 *
 * Utterance u has n_src[u] <= S sources, all of length src_len[u].  Its output
 * for mic j is y[out_off[u] + j*out_stride[u] + n], n < out_len[u], where the
 * library writes out_len[u] = T_u = src_len[u] + max_ij rir_len[r] - 1 (0 if
 * the utterance is empty) and requires out_stride[u] >= T_u.  Samples of y at
 * n >= T_u are not written.  A data array (x, h, y and the adjoint's
 * gradients of the same layouts) may be NULL when its length (x_len, h_len,
 * y_len) is 0; other NULL arguments give RSIM_EINVAL.
 */
typedef struct rsim_batch {
  int32_t n_utt;          /* U >= 0 (host) */
  int32_t n_mic;          /* J >= 1 (host) */
  int32_t max_src;        /* S >= 1 (host) */
  int32_t max_rir_len0;   /* (host) upper bound of every rir_len0 entry */
  int64_t x_len;          /* (host) floats in x: bounds for src_off + src_len */
  int64_t h_len;          /* (host) floats in h: bounds for rir_off + rir_len0 */
  int64_t y_len;          /* (host) floats in y: bounds for out_off + J*out_stride */
  const int32_t* n_src;   /* [U] */
  const int32_t* src_len; /* [U] */
  const int64_t* src_off; /* [U*S] */
  const int64_t* rir_off; /* [U*S*J] */
  const int32_t* rir_len0;/* [U*S*J] untruncated RIR lengths L0 */
  const int32_t* rir_len; /* [U*S*J] kept lengths L <= L0 (written by rsim_truncate_rir) */
  const int64_t* out_off; /* [U] */
  const int32_t* out_stride; /* [U] */
  int32_t* out_len;       /* [U] written: T_u */
  const int32_t* order;   /* [U] or NULL.  Given: the processing order, a
                           * permutation of 0..U-1 (the caller's longest-work-first
                           * order, say); with at most 65536 utterances a repeated
                           * entry is skipped and an utterance left out gets no
                           * output (T_u = 0), both with RSIM_DEV_BADDESC.  NULL:
                           * the device schedule orders each
                           * kernel family's utterances longest work first after
                           * the cut (transforms nb (I + J) + I J of the plan,
                           * weighted by N log2 N; ties in index order) in
                           * batches of up to 8192 utterances (index order in
                           * larger ones).  The order changes no output value. */
  const int32_t* fft_log2n; /* [U] or NULL: forced log2 FFT size per utterance (9..15) */
  const int32_t* hop;     /* [U] or NULL: forced block hop; default N - max L + 1 */
  int32_t fft_sizes;      /* (host) with fft_log2n: bit m set for every forced size
                           * 2^m that occurs (m = 9..15), so that only those kernel
                           * families are sized and launched; an utterance forced to
                           * a size whose bit is clear is skipped with
                           * RSIM_DEV_BADPLAN.  0: not stated, every size is
                           * provided for.  Ignored without fft_log2n. */
} rsim_batch;

/*
 * FFT-size selection table (eq. (6) and the paragraph after it: evaluate the
 * cost for each N = 2^m and keep the cheapest).  cost_fft[m-9] is the cost of
 * one real FFT of size 2^m and cost_mac[m-9] of one spectral multiply-add over
 * its N/2+1 bins; 0 disables that size.  The cost of an utterance with I
 * sources, J mics, hop B and n_b = ceil(Nx/B) blocks is
 *   n_b * ((I + J) * cost_fft + I*J * cost_mac) + I*J * cost_fft.
 * Passing NULL selects the built-in model 2.5 N log2 N / 8 (N/2+1) over all
 * sizes with one_size = 1.
 * one_size != 0 picks one N for the whole batch instead: the size with the
 * smallest cost summed over the utterances among the sizes that every
 * utterance can use (each utterance keeps its own choice if there is none).
 * Sizes forced through rsim_batch.fft_log2n take precedence over both rules.
 * variant[f] picks the work split of the filter-and-mix kernel of family f,
 * the kernels of f = 0..5 running with 32 << f threads per workgroup (N = 512;
 * 1024 and 2048; 4096; 8192; 16384; 32768):
 *   0 the library default (2); 1 one mic per pass, registers sized for two
 *   waves per SIMD; 2 two mics per pass, one wave per SIMD; 3 two mics per
 *   pass, two waves per SIMD; 4 one mic per pass, four waves per SIMD (at
 *   most 128 registers a thread, no prefetch, and one LDS exchange buffer
 *   instead of two, so that the LDS admits four waves per SIMD as well).
 *   Variants 1-3 are register budgets: with two exchange buffers (35 KB to
 *   140 KB a workgroup) the families of 256 and 512 threads hold two waves
 *   per SIMD with any of them.
 * Family 5 has variant 4 only; its entry is ignored.  Costs must be finite
 * and >= 0 and variants in 0..4 (RSIM_EINVAL, or a workspace size of 0,
 * otherwise).  The variant changes the order of no floating-point operation
 * of an output sample.  A measured table comes from autotune.py.
 */
typedef struct rsim_tune {
  float cost_fft[7];
  float cost_mac[7];
  int32_t one_size;
  int32_t variant[6];
} rsim_tune;

/* Initialise the library on the current device (twiddle tables, launch
 * geometry).  Idempotent.  Must not be called while a stream is capturing.
 * Every entry point may be called from several host threads: the library's
 * host state (per-device tables, side streams and their events, executable
 * graphs awaiting destruction) is guarded by one lock.  Device work of calls
 * on different streams is ordered only by what the caller orders, except
 * that rsim_simulate_static calls on one device share its scratch and must
 * not overlap. */
rsim_status rsim_init(void);

const char* rsim_strerror(rsim_status s);
/* 10000 major + 100 minor + patch.  The minor number changes with the layout
 * of rsim_batch or rsim_tune or with an entry point's signature (1.1:
 * rsim_batch.fft_sizes, rsim_tune.variant; 1.2: rsim_device_status takes a
 * stream); a caller built against another minor number must not call it. */
int32_t rsim_version(void);

/*
 * RIR tail cut-off, Sec. 2.3 eqs. (7)-(9), for n_rir RIRs h[off[r] .. off[r]+len0[r]).
 * Float32 rule: q[n] = fl(h[n]^2), P = max q, s = fl(10^(-eta/10)) evaluated in
 * binary64 and rounded once (eta = +inf gives s = 0), p_th = fl(P s);
 * n_c[r] = the last n with q[n] >= p_th; len[r] = min(n_c + 2, len0) (eq. (9)
 * keeps indices 0..n_c+1).  An empty RIR gives n_c = -1, len = 0; a RIR with a
 * non-finite q keeps len = len0 and sets RSIM_DEV_NONFINITE.  h_len bounds the
 * offsets (entries outside it get n_c = -1, len = 0 and RSIM_DEV_BADDESC).
 * eta_db must be >= 0 or +inf (RSIM_EINVAL otherwise).  n_c may be NULL.
 */
rsim_status rsim_truncate_rir(const float* h, int64_t h_len, const int64_t* off,
                              const int32_t* len0, int32_t n_rir, double eta_db,
                              int32_t* n_c, int32_t* len, hipStream_t stream);

/*
 * Overlap-add FFT convolution of one signal with one RIR (Sec. 2.2, eq. (6)):
 * y[0 .. nx+nh-1) = (h * x).  fft_n is a power of two in [512, 32768];
 * 1 <= hop and hop + nh - 1 <= fft_n (RSIM_EUNSUPPORTED otherwise); hop = 0
 * selects fft_n - nh + 1.  nx >= 1, nh >= 1.
 */
size_t rsim_ola_workspace_bytes(int32_t fft_n);
rsim_status rsim_ola_convolve(const float* x, int32_t nx, const float* h, int32_t nh,
                              int32_t fft_n, int32_t hop, float* y, void* ws,
                              size_t ws_bytes, hipStream_t stream);

/*
 * Batched filtering and mixing, eq. (2): for every utterance u and mic j,
 *   y_j[n] = sum_{i < n_src[u]} alpha[r] (h_r[0..rir_len[r]) * x_i)[n],
 * r = (u*S + i)*J + j, by overlap-add FFT filtering with an FFT size chosen
 * per utterance (fft_log2n, else the tune table / built-in cost model, eq. (6)).
 * alpha has U*S*J entries.  The call's kernels are a schedule kernel and one
 * persistent kernel per FFT-size family; eagerly (use_graph == 0) the family
 * kernels run concurrently on the library's side streams, forked from and
 * joined back into `stream` (one after the other when `stream` is being
 * captured).  use_graph != 0 builds them into one HIP graph, a chain (the
 * family kernels one after the other), instantiates it and launches it on
 * `stream` (which must not be capturing; the null stream is allowed).
 * ws must hold rsim_mix_workspace_bytes(b, tune, 0) bytes.
 */
size_t rsim_mix_workspace_bytes(const rsim_batch* b, const rsim_tune* tune, int32_t backward);
rsim_status rsim_mix(const rsim_batch* b, const float* x, const float* h, const float* alpha,
                     float* y, void* ws, size_t ws_bytes, const rsim_tune* tune,
                     int32_t use_graph, hipStream_t stream);

/*
 * Cut + mix of one epoch in one call: rsim_truncate_rir over every RIR slot
 * of the batch (writing b->rir_len, which must then be writable) followed by
 * rsim_mix; with use_graph != 0 all launches form one HIP graph.
 */
rsim_status rsim_simulate(const rsim_batch* b, const float* x, const float* h,
                          const float* alpha, double eta_db, int32_t* rir_len_out,
                          float* y, void* ws, size_t ws_bytes, const rsim_tune* tune,
                          int32_t use_graph, hipStream_t stream);

/*
 * For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): rsim_simulate with
 * use_graph = 0 and no workspace argument.  The workspace is a scratch array
 * of RSIM_STATIC_SCRATCH_BYTES that the library holds on each device it runs
 * on (from the library's load on that device until the process ends); the
 * call itself allocates nothing (no hipMalloc, no hipFree, no graph).  When
 * the persistent kernels' per-workgroup slots of a large batch do not all
 * fit, fewer workgroups run (same results, less parallelism); a batch whose
 * schedule arrays plus one slot per FFT-size family exceed the array is
 * rejected with RSIM_EWORKSPACE before anything is launched.  Every call on
 * a device shares that device's array and leaves its contents behind (the
 * schedule clears the work counters at the start of each call): calls that
 * overlap on one device race and give undefined results, so a caller
 * serialises them (one stream, or events).  Results are bit-identical to
 * rsim_simulate's for the same batch, eta and tune (this call never splits
 * an utterance's blocks over several work items, which keeps the scratch
 * small; the split changes no output bit).  On a capturing stream the call
 * records its kernels one after the other (no side streams, no memory set
 * or copy), so the capture can be replayed; the first call on a device must
 * come before any capture (it sets the library up).
 */
#define RSIM_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
rsim_status rsim_simulate_static(const rsim_batch* b, const float* x, const float* h,
                                 const float* alpha, double eta_db, int32_t* rir_len_out, float* y,
                                 const rsim_tune* tune, hipStream_t stream);

/*
 * Adjoint of rsim_mix (eq. (2)).  grad_y has the layout of y (only n < T_u is
 * read).  Writes
 *   grad_x[i][n]  = sum_j alpha_ij sum_{k<L_ij} h_ij[k] g_j[n+k]        (n < Nx)
 *   grad_h[r][k]  = alpha_r sum_n x_i[n] g_j[n+k]   for k < L_r, 0 for L_r <= k < L0_r
 *   grad_alpha[r] = sum_n g_j[n] (h_r * x_i)[n]     (grad_alpha may be NULL)
 * in the layouts of x, h and alpha.  The cut index gets no gradient.  Entries
 * that belong to no source or RIR slot of an utterance are not written.  The
 * FFT size and hop are chosen as by rsim_mix with the same tune.  With fewer
 * utterances than compute units, each utterance is split into block ranges:
 * a first pass forms the RIR spectra once (in ws), the parts share them, and
 * a finishing pass sums the parts' correlation spectra (in ws).  Runs eagerly
 * on `stream` and the library's side streams (as rsim_mix with use_graph 0).
 * ws must hold rsim_mix_workspace_bytes(b, tune, 1) bytes.
 */
rsim_status rsim_mix_backward(const rsim_batch* b, const float* x, const float* h,
                              const float* alpha, const float* grad_y, float* grad_x,
                              float* grad_h, float* grad_alpha, void* ws, size_t ws_bytes,
                              const rsim_tune* tune, hipStream_t stream);

/*
 * Dry power of every source slot, power[u*S + i] = mean_n x_i[n]^2 in FP64
 * (0 for unused slots), on the device.
 */
rsim_status rsim_source_power(const rsim_batch* b, const float* x, double* power,
                              hipStream_t stream);

/*
 * SNR gains of eq. (2) (host arrays): alpha[i*J + j] for I sources, J mics.
 * The paper gives no gain formula; the rule is the dry-signal SNR rule:
 * alpha_0j = 1 and alpha_ij = sqrt(p_dry[0] / (p_dry[i] 10^(snr_db[i]/10)))
 * for i >= 1 (0 if p_dry[i] <= 0), identical for every mic.
 */
rsim_status rsim_snr_gains(const double* p_dry, const double* snr_db, int32_t I, int32_t J,
                           float* alpha);

/*
 * Image-method room impulse responses, Sec. 2.1 eq. (1): the room is mirrored
 * across its walls into the (2K+1)^3 virtual rooms (a, b, c), |a|, |b|, |c| <= K
 * (K = order; the paper uses K = 8, 4913 images), each holding one image of the
 * source, and
 *   h_r[n] = sum over the images of refl^g / d,  at n = ceil(d fs / c0) < len[r],
 * g = |a| + |b| + |c| reflections, d the image-to-microphone distance, image
 * x-coordinate a Lx + xs (a even) or a Lx + (Lx - xs) (a odd), likewise y, z.
 * RIR r reads geom[9r .. 9r+9) = (Lx, Ly, Lz, source x, y, z, mic x, y, z) in
 * metres and refl[r] (device arrays, binary64) and writes every tap of
 * h[off[r] .. off[r] + len[r]).  Arithmetic in binary64 without fused
 * multiply-add: d = sqrt((dx dx + dy dy) + dz dz), n = ceil((d fs) / c0),
 * refl^g = refl multiplied g times from 1, amplitude refl^g / d; each amplitude
 * is quantised to a multiple of 2^-40 (round half to even) and the taps sum
 * these integers exactly, so the result does not depend on the order of the
 * images; a tap is then converted to binary64, scaled by 2^-40 and rounded
 * once to float32.  max_len (host) bounds every len[r].
 * Validation: n_rir >= 0, 0 <= order <= 16, fs > 0, c0 > 0, max_len >= 0
 * (RSIM_EINVAL); max_len <= 32768 (RSIM_EUNSUPPORTED).  Each RIR needs room
 * sides below 10 km, its source and microphone at least 5 mm inside every wall
 * and at least 1 cm apart (so every image is at least 1 cm from the
 * microphone and no tap's integer sum can overflow) and refl in [0, 1];
 * otherwise its taps are written as zeros and RSIM_DEV_BADDESC is set.  A
 * RIR whose taps fall outside [0, h_len) or whose len exceeds max_len is not
 * written (RSIM_DEV_BADDESC).
 */
rsim_status rsim_image_rir(const double* geom, const double* refl, int32_t n_rir, int32_t order, double fs,
                           double c0, float* h, int64_t h_len, const int64_t* off, const int32_t* len,
                           int32_t max_len, hipStream_t stream);

/*
 * One epoch with image-method rooms: rsim_image_rir into every RIR slot of
 * the batch (slot r = (u*S + i)*J + j reads geom[9r ..] and refl[r] and
 * writes h[rir_off[r] .. + rir_len0[r]); slots of length 0 are skipped, and
 * max_rir_len0 sizes the launch), then the cut and the mix of rsim_simulate
 * on those RIRs.  With use_graph != 0 the three steps form one HIP graph (a
 * chain).  Validation as rsim_simulate and rsim_image_rir (max_rir_len0 <=
 * 32768).
 */
rsim_status rsim_simulate_rooms(const rsim_batch* b, const float* x, float* h, const double* geom,
                                const double* refl, int32_t order, double fs, double c0, const float* alpha,
                                double eta_db, int32_t* rir_len_out, float* y, void* ws, size_t ws_bytes,
                                const rsim_tune* tune, int32_t use_graph, hipStream_t stream);

/*
 * Energies of the reverberant sources at the mics, for the reverberant-at-mic
 * reading of eq. (2)'s gains: energy[r] = sum_n ((h_r * x_i)[n])^2 (binary64,
 * device array of U*S*J) for RIR slot r = (u*S + i)*J + j with its kept
 * length b->rir_len[r] (call after the cut).  Computed from the identity
 * E = sum_{|l| < L} r_hh[l] r_xx[l] of the autocorrelations, in the frequency
 * domain with transforms of N = max(16384, 2^ceil(log2(2 Lmax))) points
 * (float32 transforms, binary64 sums).  Unused slots get 0; a bad descriptor NaN and RSIM_DEV_BADDESC; a
 * kept RIR longer than 16384 taps NaN and RSIM_DEV_BADPLAN.
 */
rsim_status rsim_reverb_energy(const rsim_batch* b, const float* x, const float* h, double* energy,
                               hipStream_t stream);

/*
 * Gains of the reverberant-at-mic rule (host arrays): alpha[i*J + j] from the
 * energies energy[i*J + j] of one utterance: alpha_0j = 1 and, for i >= 1,
 * alpha_ij = sqrt(E_0j / (E_ij 10^(snr_db[i]/10))), so the SNR is snr_db[i]
 * at every mic; 0 if E_ij <= 0 or E_0j <= 0.
 */
rsim_status rsim_snr_gains_reverb(const double* energy, const double* snr_db, int32_t I, int32_t J,
                                  float* alpha);

/*
 * The log-Mel front end the paper trains on (Sec. 3): for every utterance u
 * and mic j, 128 log-Mel features per frame of the output y (after rsim_mix,
 * which writes out_len): frame t covers samples [160 t, 160 t + 512) of
 * y_j, whole frames only (F_u = 1 + (out_len[u] - 512) / 160 when
 * out_len[u] >= 512); periodic Hann window; power spectrum of the 512-point
 * transform; 128 triangular filters over 130 edges equally spaced in
 * m(f) = 2595 log10(1 + f/700) from 125 to 7500 Hz; natural log of
 * (energy + 1e-6).  Frame t of (u, j) goes to
 * feat[feat_off[u] + (j C_u + t) * 128 .. + 128) with C_u the frame count of
 * out_stride[u] samples (frames t >= F_u are not written).  max_frames >=
 * every C_u (host) sizes the launch.  (Stacking four frames and keeping every
 * third, as the paper does next, is a view of these rows.)  A slot whose
 * features would leave [0, feat_len), or whose T_u is 2^29 samples or more,
 * is skipped with RSIM_DEV_BADDESC.
 */
rsim_status rsim_logmel(const rsim_batch* b, const float* y, float* feat, const int64_t* feat_off, int64_t feat_len,
                        int32_t max_frames, hipStream_t stream);

/*
 * Full-length FFT filtering, Sec. 2.2 eqs. 4-5 (the method the paper starts
 * from; overlap-add replaces it): for every utterance and mic,
 *   y_j = IFFT_N( sum_i alpha_ij FFT_N(h_ij) FFT_N(x_i) )[0, T_u),
 * N = 2^fft_log2n >= Nx + Lmax - 1 (the caller's bound for the whole batch;
 * an utterance it does not fit, or whose T_u exceeds its output stride, is
 * skipped with RSIM_DEV_BADPLAN and out_len 0), with the cut lengths in
 * b->rir_len (call after the cut).  Each transform takes two passes over
 * global memory (N = N1 N2, sub-transforms of at most 1024 points in LDS),
 * batched over `chunk` utterances at a time; ws must hold
 * rsim_fft_filter_workspace_bytes(b, fft_log2n, chunk) = 3 max_src chunk N
 * complex floats (source spectra, one mic's RIR spectra, intermediate).
 * Writes y and out_len like rsim_mix.  1 <= fft_log2n <= 20, chunk >= 1
 * (RSIM_EINVAL).
 */
size_t rsim_fft_filter_workspace_bytes(const rsim_batch* b, int32_t fft_log2n, int32_t chunk);
/*
 * The transform size of eqs. 4-5 for each utterance (host arrays, no GPU):
 * log2n[u] = ceil(log2(src_len[u] + L0max_u - 1)), L0max_u the longest
 * uncut RIR of the utterance (rir_len0[(u*max_src + i)*n_mic + j] over its
 * slots), which bounds the linear convolution for any cut; at least 1, and
 * 0 for an utterance without samples or taps.  A caller runs
 * rsim_fft_filter once per size that occurs, on the utterances of that size
 * (the descriptor's arrays are device memory, so the grouping is the
 * caller's: it needs the sizes on the host to size and launch each group).
 */
rsim_status rsim_fft_filter_sizes(const int32_t* src_len, const int32_t* rir_len0, int32_t n_utt, int32_t max_src,
                                  int32_t n_mic, int32_t* log2n);
rsim_status rsim_fft_filter(const rsim_batch* b, const float* x, const float* h, const float* alpha, float* y,
                            int32_t fft_log2n, int32_t chunk, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * One epoch with the front end fused into the mix: the cut and the mix of
 * rsim_simulate, except that the mixed samples never leave the kernels; the
 * mix kernel turns every frame of every mic output into its 128 log-Mel
 * features as soon as the frame's samples are final (Sec. 3's front end, the
 * frames, window, transform, filterbank and log of rsim_logmel, with the same
 * operations, so the features equal rsim_logmel's of rsim_simulate's
 * output when that call runs the same transform sizes).  feat, feat_off, feat_len and the frame capacity C_u (frames of
 * out_stride[u] samples) are as for rsim_logmel; y is not written (y_len,
 * out_off and out_stride keep their meaning as bounds and layout), out_len
 * is.  Only FFT sizes 4096, 8192 and 16384 have fused kernels: the size rule
 * of the tune table runs over those (one kernel variant each), and forced
 * sizes (fft_log2n) must state fft_sizes within them (RSIM_EUNSUPPORTED
 * otherwise).  Each work item keeps two overlap-add accumulators per mic in
 * its workspace slot instead of carrying through y; J <= 8
 * (RSIM_EUNSUPPORTED otherwise).  An utterance whose features would leave
 * [0, feat_len), or whose T_u is 2^29 samples or more, gets none, with
 * RSIM_DEV_BADDESC.  ws must hold rsim_simulate_logmel_workspace_bytes(b,
 * tune) bytes; use_graph as for rsim_simulate.
 */
size_t rsim_simulate_logmel_workspace_bytes(const rsim_batch* b, const rsim_tune* tune);
rsim_status rsim_simulate_logmel(const rsim_batch* b, const float* x, const float* h, const float* alpha,
                                 double eta_db, int32_t* rir_len_out, float* feat, const int64_t* feat_off,
                                 int64_t feat_len, void* ws, size_t ws_bytes, const rsim_tune* tune,
                                 int32_t use_graph, hipStream_t stream);

/* Waits for the work queued on `stream` (which includes the library's side
 * streams of every call made on it), then reads the current device's status
 * word into *status (host) and clears it.  Flags that kernels still running
 * on other streams set after the read are kept for the next read; one set
 * between the read and the clear is lost, so read it when the device's other
 * streams are idle.  RSIM_EDEVICE if the stream or a copy fails. */
rsim_status rsim_device_status(hipStream_t stream, int32_t* status);

/*
 * Transform entry points of the FFT engine, for its unit tests: `count` real
 * signals of length n (power of two, 512..32768), contiguous.  rsim_rfft
 * writes n/2+1 complex bins per signal (interleaved float pairs), unscaled;
 * rsim_irfft is its inverse (scaled by 1/n), reading n/2+1 bins.
 */
rsim_status rsim_rfft(const float* x, int32_t n, int32_t count, float* spec, hipStream_t stream);
rsim_status rsim_irfft(const float* spec, int32_t n, int32_t count, float* x, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* RSIM_H */

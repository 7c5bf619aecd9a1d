// Device kernels of the room-simulator hot path: RIR cut-off (Sec. 2.3,
// eqs. 7-9), per-utterance FFT-size schedule (eq. 6), and the persistent
// overlap-add filter-and-mix kernel (Sec. 2.2 eq. 6 applied to eq. 2).
#pragma once

#include "fft_engine.hpp"

namespace rsim {

// Twiddle tables of every plan (filled from FP64 host values at init) and the
// per-device status word.
extern __device__ cf g_tw[kTwTotal];
extern __device__ int g_status;

// Kernel families, one per workgroup size T = 32 << f (f = 0..5): every
// FFT size runs in the family of its plan's thread count.
constexpr int kNumFam = 6;

__host__ __device__ constexpr int family_of_log2n(int l2) {
  return ilog2c(plan_threads(l2)) - 5;
}

// Per-utterance plan written by the schedule kernel.
struct Sched {
  int log2n;  // FFT size N = 2^log2n (0 if the utterance is skipped)
  int hop;    // block hop B
  int nb;     // number of blocks ceil(Nx / B)
  int tu;     // output length Nx + Lmax - 1
  int lmax;   // max kept RIR length over the utterance
  int pad_;
};

struct BatchDev {
  int U, J, S;
  long long x_len, h_len, y_len;
  const int* n_src;
  const int* src_len;
  const long long* src_off;
  const long long* rir_off;
  const int* rir_len0;
  const int* rir_len;
  const long long* out_off;
  const int* out_stride;
  int* out_len;
  const int* order;
  const int* fft_log2n;
  const int* hop;
  int fft_sizes;  // bit m: forced size 2^m provided for; 0 = every size
};

struct TuneDev {
  float cost_fft[7];
  float cost_mac[7];
  int one_size;
  int variant[kNumFam];  // host side only: kernel variant of each family (0..3)
};

// Workspace header shared by the schedule and mix launches of one call.
struct WsHeader {
  int counter[kNumFam];  // work-queue heads
  int count[kNumFam];    // items per family
};

struct MixArgs {
  BatchDev b;
  const float* x;
  const float* h;
  const float* alpha;
  float* y;
  const Sched* sched;
  const int* list;  // this family's utterances, in processing order
  WsHeader* hdr;
  int fam;
  cf* scratch;          // per-workgroup scratch base
  long long slot_cf;    // complex entries per workgroup
  // 1: a work item is an utterance; g > 1 (batches with few utterances): a
  // work item is one mic group of an utterance, g items per utterance.
  int gsplit;
  // psplit > 1 (batches with fewer work items than compute units): each
  // (utterance, mic group) is further split into up to psplit block ranges
  // (parts).  The alpha-scaled RIR spectra of the family's utterances are
  // then formed once by a pass before the kernel, into hspec
  // ([U][S J][mmax], mmax the family's largest M); the first block of a part
  // p > 0 leaves the head of its output (the samples the previous block's
  // tail also covers) in seam ([U][psplit][J][mmax] floats) instead of y,
  // and a pass after the kernel adds it to y.
  int psplit;
  int mmax;
  cf* hspec;
  float* seam;
  // The front end fused into the mix (mix kernels built with it): the
  // 128-band log-Mel features of every mic output go to feat (the layout of
  // rsim_logmel) instead of the samples to y; each workgroup's slot then also
  // holds two overlap-add accumulators per mic (2M complex entries a mic).
  float* feat;
  const long long* feat_off;
  long long feat_len;
};

struct BwdArgs {
  BatchDev b;
  const float* x;
  const float* h;
  const float* alpha;
  const float* gy;
  float* gx;
  float* gh;
  float* galpha;
  const Sched* sched;
  const int* list;
  WsHeader* hdr;
  int fam;
  cf* scratch;
  long long slot_cf;
  // Splitting of an utterance over several work items (for batches with few
  // utterances): item (u, r), r < nsplit, covers a range of u's blocks and
  // accumulates its share of the correlation spectra in `partial`
  // ([U][nsplit][S J][mmax], mmax the family's largest M: the sizes of one
  // family differ); a finishing pass sums them.
  int nsplit;
  int mmax;
  cf* partial;
  // With nsplit > 1, the alpha-scaled RIR spectra of every utterance of the
  // family, formed once by a pass before the parts ([U][S J][mmax]).
  cf* hspec;
};

}  // namespace rsim

// librsim: HIP kernels for gfx950 and the C ABI declared in include/rsim.h.
//
// Hot path (one call of rsim_mix / rsim_simulate):
//   truncate_kernel  RIR tail cut-off, Sec. 2.3 eqs. (7)-(9)
//   prepare_kernel   per utterance, in parallel: descriptor checks, longest
//                    kept RIR, cost of every FFT size N = 2^m (eq. (6))
//   schedule_kernel  FFT size / hop / block count per utterance (one size for
//                    the batch or each its own, as the text after eq. (6)
//                    chooses per filtering), lists per workgroup size in the
//                    caller's order or, without one, longest work first
//   mix_kernel<T>    persistent workgroups pop work items (an utterance, or
//                    one mic group of it, or a range of its blocks); each
//                    computes the RIR spectra once (Sec. 2.2: the RIR FFT is
//                    not repeated per block), then walks the blocks: FFT of
//                    each source block, spectral multiply-accumulate over
//                    sources per mic, inverse FFT, overlap-add (eq. (6)) into
//                    y (eq. (2)).  With block ranges, mix_rir_kernel<T> forms
//                    the RIR spectra first and mix_seam_kernel adds the seams.
// Adjoint (rsim_mix_backward): bwd_kernel<T> per utterance or block range,
// bwd_rir_kernel<T> and bwd_finish_kernel<T> for split utterances,
// bwd_zero_kernel for idle ones.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <vector>

#include "../../include/rsim.h"
#include "kernels.hpp"

namespace rsim {

__device__ cf g_tw[kTwTotal];
__device__ int g_status;
// Log-Mel front end: periodic Hann window of 512 samples and the 128
// triangular Mel filters over the 257 bins of a 512-point transform (bands
// as bin ranges with their weights), filled at init from binary64 values.
constexpr int kMelWin = 512, kMelHop = 160, kMelBands = 128, kMelBins = kMelWin / 2 + 1;
// Nonzero weights of a band, at most, for bands 0-31, 32-63, 64-95, 96-127
// (the triangles widen with frequency: 2, 3, 6 and 9 bins for this scale).
constexpr int kMelCap0 = 3, kMelCap1 = 4, kMelCap2 = 7, kMelCap3 = 10, kMelCapMax = 10;
__device__ __host__ constexpr int mel_cap(int quarter) {
  return quarter == 0 ? kMelCap0 : quarter == 1 ? kMelCap1 : quarter == 2 ? kMelCap2 : kMelCap3;
}
__device__ float g_hann[kMelWin];
__device__ int g_mel_first[kMelBands];
__device__ float g_mel_w[kMelBands * kMelCapMax];  // band b's weights at [b * kMelCapMax, + count), zero after

constexpr int kMelMaxT = 1 << 29;  // mic signals shorter than this (byte offsets fit 31 bits)
// Whole frames in T samples.
__device__ __forceinline__ int mel_frames(int T) { return T >= kMelWin ? 1 + (T - kMelWin) / kMelHop : 0; }

// Band energy sum_i w[i] pw[first + i] over i < CAP, in bin order; the
// weights past the band's bins are zero, so for finite powers those terms
// add exactly nothing.  (A non-finite power can also make the bands whose
// padded range covers it NaN; with the full filterbank matrix it makes
// every band NaN.)
template <int CAP>
__device__ __forceinline__ float mel_band(const float* w, const float* pw, int first) {
  float p[CAP];
#pragma unroll
  for (int i = 0; i < CAP; ++i) p[i] = pw[first + i];
  float m = 0.f;
#pragma unroll
  for (int i = 0; i < CAP; ++i) m = __builtin_fmaf(w[i], p[i], m);
  return m;
}

__device__ __forceinline__ void flag_status(int bits) { atomicOr(&g_status, bits); }

// Values that are the same in every lane (descriptor entries of the current
// utterance): keeping them in scalar registers keeps the buffer resources
// built from them scalar.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long long uni64(long long v) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(v & 0xffffffffLL));
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((unsigned long long)v >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}

// ------------------------------------------------------------------ reductions
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v |= __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// =============================================================== RIR cut-off
// One wave per RIR (four per workgroup), no workgroup barrier: each lane
// reads four consecutive taps per step (one 128-bit access; the range check
// zero-fills past L0).  P = max_n fl(h^2) by a max-reduction (exact in any
// order), p_th = fl(P s), then the last index with q >= p_th, searched 256
// taps at a time from the tail, so only the part behind the cut is read
// twice (the second time from cache).
constexpr int kTruncThreads = 256;
constexpr int kTruncWaves = kTruncThreads / 64;

struct TruncArgs {
  const float* h;
  long long h_len;
  const long long* off;
  const int* len0;
  int n_rir;
  float s;     // fl32(10^(-eta/10)), 0 for eta = inf
  int* n_c;    // may be null
  int* len;
};

// Chunks of 1024 taps whose maxima a wave keeps in LDS (RIRs up to 32768
// taps); past that the tail search reads the taps again, 256 at a time.
constexpr int kTruncChunks = 32;

__global__ __launch_bounds__(kTruncThreads) void truncate_kernel(TruncArgs A) {
  __shared__ float s_cmax[kTruncWaves][kTruncChunks];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int r0 = blockIdx.x * kTruncWaves; r0 < A.n_rir; r0 += gridDim.x * kTruncWaves) {
    const int r = r0 + w;
    if (r >= A.n_rir) continue;
    const int L0 = uni(A.len0[r]);
    const long long o = uni64(A.off[r]);
    if (L0 < 0 || o < 0 || o + (long long)L0 > A.h_len) {
      if (lane == 0) {
        flag_status(RSIM_DEV_BADDESC);
        if (A.n_c) A.n_c[r] = -1;
        A.len[r] = 0;
      }
      continue;
    }
    if (L0 == 0) {
      if (lane == 0) {
        if (A.n_c) A.n_c[r] = -1;
        A.len[r] = 0;
      }
      continue;
    }
    const rsrc_t rs = make_rsrc(A.h + o, L0 * 4);
    const int vo = 16 * lane;
    // max pass: four chunks of 1024 taps per step, sixteen 128-bit loads in
    // flight per lane; each chunk's maximum is kept for the tail search
    float mx = 0.0f;
    int nf = 0;
    for (int base = 0, c = 0; base < L0; base += 4096, c += 4) {
      f4 v[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) v[k] = ld4(rs, vo + 4 * (base + 256 * k));  // whole offset range-checked
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        float cm = 0.0f;
#pragma unroll
        for (int k = 4 * cc; k < 4 * cc + 4; ++k) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float q = v[k][e] * v[k][e];
            nf |= !__builtin_isfinite(q);
            cm = fmaxf(cm, q);
          }
        }
        mx = fmaxf(mx, cm);
        if (c + cc < kTruncChunks) {
          cm = wave_max(cm);
          if (lane == 0) s_cmax[w][c + cc] = cm;
        }
      }
    }
    mx = wave_max(mx);
    nf = wave_or(nf);
    if (nf) {
      if (lane == 0) {
        flag_status(RSIM_DEV_NONFINITE);
        if (A.n_c) A.n_c[r] = L0 - 1;
        A.len[r] = L0;
      }
      continue;
    }
    const float pth = mx * A.s;
    const int nch = (L0 + 1023) / 1024;
    int found = -1;
    if (nch <= kTruncChunks) {
      // the last chunk whose maximum reaches p_th holds the last such tap
      // (wave-local LDS: the wave wrote these values itself)
      const bool hit = lane < nch && s_cmax[w][lane] >= pth;
      const unsigned long long m = __ballot(hit);
      const int c = m ? 63 - __builtin_clzll(m) : 0;
      const int base = c * 1024;
      f4 v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = ld4(rs, vo + 4 * (base + 256 * k));
      int loc = -1;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int idx = base + 256 * k + 4 * lane + e;
          if (idx < L0 && v[k][e] * v[k][e] >= pth) loc = idx;
        }
      }
      found = wave_max_i(loc);
    } else {
      for (int base = ((L0 - 1) / 256) * 256; base >= 0; base -= 256) {
        const f4 v = ld4(rs, vo + 4 * base);  // whole offset range-checked
        int loc = -1;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int idx = base + 4 * lane + k;
          if (idx < L0 && v[k] * v[k] >= pth) loc = idx;
        }
        loc = wave_max_i(loc);
        if (loc >= 0) {
          found = loc;
          break;
        }
      }
    }
    if (lane == 0) {
      if (A.n_c) A.n_c[r] = found;
      A.len[r] = min(found + 2, L0);
    }
  }
}

// ================================================================= schedule
// Validates utterance u's descriptor and returns its longest kept RIR
// (0: nothing to write); -1 (with err set) for a bad descriptor.
__device__ int utterance_lmax(const BatchDev& b, int u, int& err) {
  const int I = b.n_src[u], Nx = b.src_len[u], J = b.J;
  if (I < 0 || I > b.S || Nx < 0) {
    err |= RSIM_DEV_BADDESC;
    return -1;
  }
  int lmax = 0;
  for (int i = 0; i < I; ++i) {
    const long long so = b.src_off[(long long)u * b.S + i];
    if (so < 0 || so + Nx > b.x_len) {
      err |= RSIM_DEV_BADDESC;
      return -1;
    }
    for (int j = 0; j < J; ++j) {
      const long long r = ((long long)u * b.S + i) * J + j;
      const int L0 = b.rir_len0[r], L = b.rir_len[r];
      const long long ro = b.rir_off[r];
      if (L < 0 || L > L0 || ro < 0 || ro + L0 > b.h_len) {
        err |= RSIM_DEV_BADDESC;
        return -1;
      }
      lmax = max(lmax, L);
    }
  }
  if (I == 0 || Nx == 0 || lmax == 0) return 0;  // nothing to write
  const long long tu = (long long)Nx + lmax - 1;
  const long long ys = b.out_stride[u], yo = b.out_off[u];
  if (tu > 0x7fffffffLL || ys < tu || yo < 0 || yo + (long long)J * ys > b.y_len) {
    err |= RSIM_DEV_BADDESC;
    return -1;
  }
  return lmax;
}

// Cost of utterance u at N = 2^m under the tune table (eq. 6's rule with the
// kernel's transform count); negative when N cannot serve it.
__device__ float utterance_cost(const BatchDev& b, const TuneDev& tune, int u, int lmax, int m) {
  const float cf_ = tune.cost_fft[m - 9], cm = tune.cost_mac[m - 9];
  if (!(cf_ > 0.f)) return -1.f;
  const int N = 1 << m;
  if (N < lmax) return -1.f;
  const int given_hop = b.hop ? b.hop[u] : 0;
  const int B = given_hop ? given_hop : N - lmax + 1;
  if (B < 1 || B + lmax - 1 > N) return -1.f;
  const int I = b.n_src[u], Nx = b.src_len[u], J = b.J;
  const float nbf = (float)((Nx + B - 1) / B);
  return nbf * ((float)(I + J) * cf_ + (float)(I * J) * cm) + (float)(I * J) * cf_;
}

// The plan of utterance u with longest kept RIR lmax (> 0): the forced size
// if the descriptor gives one, else `batch_l2` if nonzero (one size for the
// whole batch), else its cheapest size.
__device__ Sched plan_utterance(const BatchDev& b, const TuneDev& tune, int u, int lmax, int batch_l2, int& err) {
  Sched S = {0, 0, 0, 0, 0, 0};
  if (lmax <= 0) return S;
  const int Nx = b.src_len[u];
  const long long tu = (long long)Nx + lmax - 1;
  const int given_hop = b.hop ? b.hop[u] : 0;
  int l2 = 0;
  if (b.fft_log2n) {
    l2 = b.fft_log2n[u];
    // a forced size outside the stated set has no kernel family launched
    if (b.fft_sizes && l2 >= 9 && l2 <= 15 && !((b.fft_sizes >> l2) & 1)) l2 = 0;
  } else if (batch_l2) {
    l2 = batch_l2;
  } else {
    float best = 0.f;
    for (int m = 9; m <= 15; ++m) {
      const float cost = utterance_cost(b, tune, u, lmax, m);
      if (cost < 0.f) continue;
      if (l2 == 0 || cost < best) {
        best = cost;
        l2 = m;
      }
    }
  }
  if (l2 < 9 || l2 > 15) {
    err |= RSIM_DEV_BADPLAN;
    return S;
  }
  const int N = 1 << l2;
  const int B = given_hop ? given_hop : N - lmax + 1;
  if (B < 1 || B + lmax - 1 > N) {
    err |= RSIM_DEV_BADPLAN;
    return S;
  }
  S.log2n = l2;
  S.hop = B;
  S.nb = (Nx + B - 1) / B;
  S.tu = (int)tu;
  S.lmax = lmax;
  return S;
}

struct SchedArgs {
  BatchDev b;
  TuneDev tune;
  Sched* sched;
  int* lists;
  WsHeader* hdr;
  float* costs;  // [U][8]: per-size costs of each utterance (one size per batch)
};

// First step of the schedule, over every utterance in parallel: validates
// its descriptor, records its longest kept RIR (or -1 for a bad descriptor)
// in its plan slot and, for one size per batch, its cost at every size
// (negative: that size cannot serve it).
constexpr int kPrepThreads = 256;
__global__ __launch_bounds__(kPrepThreads) void prepare_kernel(SchedArgs A) {
  const BatchDev& b = A.b;
  int err = 0;
  for (int u = blockIdx.x * kPrepThreads + threadIdx.x; u < b.U; u += gridDim.x * kPrepThreads) {
    const int lmax = utterance_lmax(b, u, err);
    Sched S = {0, 0, 0, 0, lmax, 0};
    A.sched[u] = S;
    if (A.tune.one_size && !b.fft_log2n) {
      for (int m = 9; m <= 15; ++m) A.costs[(long long)u * 8 + m - 9] = lmax > 0 ? utterance_cost(b, A.tune, u, lmax, m) : 0.f;
    }
  }
  if (err) flag_status(err);
}

// One workgroup of 1024 threads: plans every utterance and appends it to its
// family's list in the caller's order (a stable compaction per family).
// Without a caller's order, in batches of up to kLptCap utterances, each list
// is then sorted longest work first (LPT): by decreasing transform count
// nb (I + J) + I J of the utterance's plan, weighted by N log2 N (one family
// can hold two sizes), ties in utterance order.  The 32-bit key of list
// position k is the work's float bits without their 13 lowest (positive
// floats order as their bits; the rest keeps a relative resolution of 2^-10,
// ample for an order of work), then kLptCap - 1 - k, so the earlier position
// comes first among equal work.  Each thread keeps the position, family and
// work of the (at most kLptChunks) utterances it planned in registers, and a
// bitonic network sorts each list: its stages with a stride of at most 64
// exchange within 128 entries, which one wave holds in registers (two per
// lane) and exchanges by lane shuffles; the longer strides go through LDS.
// Larger batches keep index order.
constexpr int kSchedThreads = 1024;
constexpr int kLptBits = 13, kLptCap = 1 << kLptBits, kLptChunks = kLptCap / kSchedThreads;
constexpr int kSeenBits = 65536;  // utterances whose caller's order is checked

// The stages of sizes `size` (strides smax .. 1, smax <= 64) of the bitonic
// network (descending where bit `size` of the index is clear) on one wave's
// block of 128 entries held in registers: lane l holds entries i0 = 2 l and
// i0 + 1 of the block (whose index bits above 7 are i0's).  Stride 1 pairs a
// lane's own two entries; stride s >= 2 pairs lane l with lane l ^ (s / 2).
__device__ __forceinline__ void lpt_wave_stages(unsigned& e0, unsigned& e1, int i0, int lane, int size, int smax) {
  for (int s = smax; s >= 1; s >>= 1) {
    const bool desc = (i0 & size) == 0;  // bit `size` lies above s: the same for both entries
    if (s == 1) {
      const unsigned a = e0, c = e1;
      const bool swap = desc ? a < c : a > c;
      e0 = swap ? c : a;
      e1 = swap ? a : c;
    } else {
      const int m = s >> 1;
      const unsigned p0 = __shfl_xor(e0, m), p1 = __shfl_xor(e1, m);
      const bool take_max = ((lane & m) == 0) == desc;  // the lower index keeps the larger key when descending
      e0 = take_max ? max(e0, p0) : min(e0, p0);
      e1 = take_max ? max(e1, p1) : min(e1, p1);
    }
  }
}

// Sorts list f (n entries) given each thread's records: chunk c of thread t
// is utterance c * kSchedThreads + t, at position pos[c] of list fam[c] with
// work prefix wk[c].
__device__ void lpt_sort_list(int* __restrict__ lf, int f, int n, const int* fam, const int* pos,
                              const unsigned* wk, unsigned* s_key, int* s_u, int t) {
  int p2 = 128;
  while (p2 < n) p2 <<= 1;
  for (int k = n + t; k < p2; k += kSchedThreads) s_key[k] = 0u;  // padding: below every real key
#pragma unroll
  for (int c = 0; c < kLptChunks; ++c) {
    if (fam[c] == f) {
      s_key[pos[c]] = wk[c] | (unsigned)(kLptCap - 1 - pos[c]);
      s_u[pos[c]] = c * kSchedThreads + t;
    }
  }
  __syncthreads();
  // Strides of at most 64 run in registers, one wave per block of 128
  // entries; the longer ones go through LDS with workgroup barriers.
  const int lane = t & 63, wv = t >> 6, nblk = p2 >> 7;
  for (int wb = wv; wb < nblk; wb += kSchedThreads / 64) {
    const int i0 = 128 * wb + 2 * lane;
    unsigned e0 = s_key[i0], e1 = s_key[i0 + 1];
    for (int size = 2; size <= 128; size <<= 1) lpt_wave_stages(e0, e1, i0, lane, size, size >> 1);
    s_key[i0] = e0;
    s_key[i0 + 1] = e1;
  }
  __syncthreads();
  for (int size = 256; size <= p2; size <<= 1) {
    for (int stride = size >> 1; stride >= 128; stride >>= 1) {
      for (int k = t; k < p2 / 2; k += kSchedThreads) {
        const int lo = 2 * k - (k & (stride - 1)), hi = lo + stride;
        const bool desc = (lo & size) == 0;  // the final merge (size = p2) is descending throughout
        const unsigned a = s_key[lo], c = s_key[hi];
        if (desc ? a < c : a > c) {
          s_key[lo] = c;
          s_key[hi] = a;
        }
      }
      __syncthreads();
    }
    for (int wb = wv; wb < nblk; wb += kSchedThreads / 64) {
      const int i0 = 128 * wb + 2 * lane;
      unsigned e0 = s_key[i0], e1 = s_key[i0 + 1];
      lpt_wave_stages(e0, e1, i0, lane, size, 64);
      s_key[i0] = e0;
      s_key[i0 + 1] = e1;
    }
    __syncthreads();
  }
  for (int k = t; k < n; k += kSchedThreads) lf[k] = s_u[kLptCap - 1 - (int)(s_key[k] & (kLptCap - 1))];
  __syncthreads();
}

__global__ __launch_bounds__(kSchedThreads) void schedule_kernel(SchedArgs A) {
  const BatchDev& b = A.b;
  const TuneDev& tune = A.tune;
  Sched* __restrict__ sched = A.sched;
  int* __restrict__ lists = A.lists;
  WsHeader* hdr = A.hdr;
  __shared__ int s_wcnt[kNumFam][kSchedThreads / 64];
  __shared__ int s_base[kNumFam];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  if (t < kNumFam) {
    hdr->counter[t] = 0;
    s_base[t] = 0;
  }
  int err = 0;
  // One size for the whole batch: the size with the smallest cost summed over
  // the utterances, among the sizes every utterance with work can use.
  __shared__ double s_cost[7];
  __shared__ int s_bad[7];
  __shared__ int s_l2;
  int batch_l2 = 0;
  if (tune.one_size && !b.fft_log2n) {
    if (t < 7) {
      s_cost[t] = 0.0;
      s_bad[t] = 0;
    }
    __syncthreads();
    for (int c0 = 0; c0 < b.U; c0 += kSchedThreads) {
      const int u = c0 + t;
      const int lmax = u < b.U ? sched[u].lmax : 0;
      for (int m = 9; m <= 15; ++m) {
        const float c = lmax > 0 ? A.costs[(long long)u * 8 + m - 9] : 0.f;
        const double cs = wave_sum_d(c > 0.f ? (double)c : 0.0);
        const int bad = wave_or(lmax > 0 && c < 0.f);
        if ((t & 63) == 0) {
          atomicAdd(&s_cost[m - 9], cs);
          if (bad) atomicOr(&s_bad[m - 9], 1);
        }
      }
    }
    __syncthreads();
    if (t == 0) {
      int best = 0;
      for (int m = 9; m <= 15; ++m)
        if (!s_bad[m - 9] && tune.cost_fft[m - 9] > 0.f && (best == 0 || s_cost[m - 9] < s_cost[best - 9]))
          best = m;
      s_l2 = best;  // 0: no common size, each utterance takes its own
    }
    __syncthreads();
    batch_l2 = s_l2;
  }
  __syncthreads();
  // A caller's order must be a permutation: with up to kSeenBits utterances a
  // bitmap in LDS finds repeated entries (skipped, flagged) and utterances the
  // order leaves out (no output, flagged).
  __shared__ unsigned s_seen[kSeenBits / 32];
  const bool check_order = b.order && b.U <= kSeenBits;
  if (check_order) {
    for (int k = t; k < kSeenBits / 32; k += kSchedThreads) s_seen[k] = 0u;
    __syncthreads();
  }
  // Plans the utterances of list positions c0 .. c0 + kSchedThreads - 1 and
  // appends them to their families' lists; returns this thread's family (-1:
  // none), its list position and the prefix of its sort key.
  auto plan_chunk = [&](int c0, int& pos, unsigned& wk) __attribute__((always_inline)) {
    const int idx = c0 + t;
    int fam = -1, u = -1;
    Sched S = {0, 0, 0, 0, 0, 0};
    if (idx < b.U) {
      u = b.order ? b.order[idx] : idx;
      bool dup = false;
      if (b.order && u >= 0 && u < b.U && check_order) {
        const unsigned bit = 1u << (u & 31);
        dup = (atomicOr(&s_seen[u >> 5], bit) & bit) != 0;
      }
      if (u < 0 || u >= b.U || dup) {
        err |= RSIM_DEV_BADDESC;
        u = -1;
      } else {
        S = plan_utterance(b, tune, u, sched[u].lmax, batch_l2, err);
        sched[u] = S;
        b.out_len[u] = S.tu;
        fam = S.nb > 0 ? family_of_log2n(S.log2n) : -1;
      }
    }
    if (fam >= 0) {
      const int I = b.n_src[u];
      const float work = ((float)S.nb * (float)(I + b.J) + (float)(I * b.J)) * (float)((1 << S.log2n) * S.log2n);
      wk = (__float_as_uint(work) >> kLptBits) << kLptBits;
    }
    int pre[kNumFam];
#pragma unroll
    for (int f = 0; f < kNumFam; ++f) {
      const unsigned long long m = __ballot(fam == f);
      pre[f] = __popcll(m & ((1ull << lane) - 1ull));
      if (lane == 0) s_wcnt[f][w] = __popcll(m);
    }
    __syncthreads();
#pragma unroll
    for (int f = 0; f < kNumFam; ++f) {
      if (fam == f) {
        int o = s_base[f];
        for (int k = 0; k < w; ++k) o += s_wcnt[f][k];
        pos = o + pre[f];
        lists[(long long)f * b.U + pos] = u;
      }
    }
    __syncthreads();
    if (t < kNumFam) {
      int tot = 0;
      for (int k = 0; k < kSchedThreads / 64; ++k) tot += s_wcnt[t][k];
      s_base[t] += tot;
    }
    __syncthreads();
    return fam;
  };
  const bool lpt = !b.order && b.U <= kLptCap;
  int r_fam[kLptChunks], r_pos[kLptChunks];
  unsigned r_wk[kLptChunks];
#pragma unroll
  for (int c = 0; c < kLptChunks; ++c) {
    r_fam[c] = -1;
    r_pos[c] = 0;
    r_wk[c] = 0u;
    if (c * kSchedThreads < b.U) r_fam[c] = plan_chunk(c * kSchedThreads, r_pos[c], r_wk[c]);
  }
  for (int c0 = kLptChunks * kSchedThreads; c0 < b.U; c0 += kSchedThreads) {
    int pos = 0;
    unsigned wk = 0u;
    plan_chunk(c0, pos, wk);
  }
  if (t < kNumFam) hdr->count[t] = s_base[t];
  if (check_order) {
    for (int u = t; u < b.U; u += kSchedThreads) {
      if (!(s_seen[u >> 5] & (1u << (u & 31)))) {
        const Sched none = {0, 0, 0, 0, 0, 0};
        sched[u] = none;
        b.out_len[u] = 0;
        err |= RSIM_DEV_BADDESC;
      }
    }
  }
  if (lpt) {
    __shared__ unsigned s_key[kLptCap];
    __shared__ int s_u[kLptCap];
    for (int f = 0; f < kNumFam; ++f) {
      const int n = s_base[f];
      if (n >= 2) lpt_sort_list(lists + (long long)f * b.U, f, n, r_fam, r_pos, r_wk, s_key, s_u, t);
    }
  }
  if (err) flag_status(err);
}

// ============================================================ filter and mix
// v[r] = (src[2(t + rT)], src[2(t + rT) + 1]), zero at indices >= nvalid
// (the buffer range check supplies the zero padding of the block).
template <class PL>
__device__ __forceinline__ void load_real(cf* v, const float* __restrict__ src, int nvalid, int t_) {
  const int t = opaque_v(t_);
  const rsrc_t rs = make_rsrc(src, nvalid * 4);
  const int vo = 8 * t;
#pragma unroll
  for (int r = 0; r < PL::P; ++r) v[r] = ld2(rs, vo + 8 * r * PL::T);
}

// Spectra in memory: slot q of thread t at index q * T + t.
template <class PL>
__device__ __forceinline__ void store_spec(cf* __restrict__ dst, const cf* v, int t) {
  const rsrc_t rs = make_rsrc(dst, PL::P * PL::T * 8);
  const int vo = 8 * opaque_v(t);
#pragma unroll
  for (int q = 0; q < PL::P; ++q) st2(rs, vo, v[q], 8 * q * PL::T);
}

template <class PL>
__device__ __forceinline__ void load_spec(cf* v, const cf* __restrict__ src, int t) {
  const rsrc_t rs = make_rsrc(src, PL::P * PL::T * 8);
  const int vo = 8 * opaque_v(t);
#pragma unroll
  for (int q = 0; q < PL::P; ++q) v[q] = ld2(rs, vo, 8 * q * PL::T);
}

// Bin held by slot q of thread t (thread 0 permuted as in Fft::perm_t0; its
// slot SP holds bins 0 and N/2).
template <class PL>
__device__ __forceinline__ int slot_bin(int q, int t) {
  constexpr int R = PL::RL, T = PL::T;
  if (t != 0) return q < R ? t + 2 * T * q : (2 * T - t) + 2 * T * (q - R);
  if (q < R / 2) return T + 2 * T * q;
  if (q < R) return 2 * T * q;
  if (q < 3 * R / 2 - 1) return 2 * T * (q - R + 1);
  if (q == 3 * R / 2 - 1) return 0;
  return T + 2 * T * (q - R);
}

// The mix kernel's RIR spectra in pairs: slots 2p, 2p + 1 of thread t at
// index p 2T + 2t, so one 128-bit access moves both (half the load
// instructions of the slot layout for the same bytes).
template <class PL>
__device__ __forceinline__ void store_spec_pair(cf* __restrict__ dst, const cf* v, int t) {
  static_assert(PL::P % 2 == 0, "slots come in pairs");
  const rsrc_t rs = make_rsrc(dst, PL::P * PL::T * 8);
  const int vo = 16 * opaque_v(t);
  typedef unsigned u4 __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int p = 0; p < PL::P / 2; ++p) {
    const f4 w = {v[2 * p].x, v[2 * p].y, v[2 * p + 1].x, v[2 * p + 1].y};
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, w), rs, vo, 16 * p * PL::T, 0);
  }
}
template <class PL>
__device__ __forceinline__ void load_spec_pair(cf* v, const cf* __restrict__ src, int t) {
  const rsrc_t rs = make_rsrc(src, PL::P * PL::T * 8);
  const int vo = 16 * opaque_v(t);
#pragma unroll
  for (int p = 0; p < PL::P / 2; ++p) {
    const f4 w = ld4(rs, vo, 16 * p * PL::T);
    v[2 * p] = mk(w.x, w.y);
    v[2 * p + 1] = mk(w.z, w.w);
  }
}

// Y += H X over the thread's slots (H in the paired layout); thread 0's slot SP is the packed pair of
// real bins (0, N/2) and multiplies componentwise.
template <class PL>
__device__ __forceinline__ void mac(cf* Y, const cf* __restrict__ H, const cf* X, int t_) {
  constexpr int SP = Fft<PL>::SP;
  const int t = opaque_v(t_);
  const rsrc_t rs = make_rsrc(H, PL::P * PL::T * 8);
  const int vo = 16 * t;
  f4 w;
#pragma unroll
  for (int q = 0; q < PL::P; ++q) {
    if ((q & 1) == 0) w = ld4(rs, vo, 16 * (q >> 1) * PL::T);  // slots q, q + 1
    const cf hv = (q & 1) ? mk(w.z, w.w) : mk(w.x, w.y);
    if (q == SP) {
      const cf c = cmac(Y[q], hv, X[q]);
      const cf d = mk(__builtin_fmaf(hv.x, X[q].x, Y[q].x), __builtin_fmaf(hv.y, X[q].y, Y[q].y));
      Y[q] = t == 0 ? d : c;
    } else {
      Y[q] = cmac(Y[q], hv, X[q]);
    }
  }
}

// Y += H X with H already in registers.
template <class PL>
__device__ __forceinline__ void mac_regs(cf* Y, const cf* Hr, const cf* X, int t_) {
  constexpr int SP = Fft<PL>::SP;
  const int t = opaque_v(t_);
#pragma unroll
  for (int q = 0; q < PL::P; ++q) {
    const cf hv = Hr[q];
    if (q == SP) {
      const cf c = cmac(Y[q], hv, X[q]);
      const cf d = mk(__builtin_fmaf(hv.x, X[q].x, Y[q].x), __builtin_fmaf(hv.y, X[q].y, Y[q].y));
      Y[q] = t == 0 ? d : c;
    } else {
      Y[q] = cmac(Y[q], hv, X[q]);
    }
  }
}

// Two mics at once: Y0 += H0 X, Y1 += H1 X, one slot at a time (H paired).
template <class PL>
__device__ __forceinline__ void mac2(cf* Y0, cf* Y1, const cf* __restrict__ H0,
                                     const cf* __restrict__ H1, const cf* X, int t_) {
  constexpr int SP = Fft<PL>::SP;
  const int t = opaque_v(t_);
  const rsrc_t r0 = make_rsrc(H0, PL::P * PL::T * 8);
  const rsrc_t r1 = make_rsrc(H1, PL::P * PL::T * 8);
  const int vo = 16 * t;
  f4 w0, w1;
#pragma unroll
  for (int q = 0; q < PL::P; ++q) {
    if ((q & 1) == 0) {  // slots q, q + 1
      w0 = ld4(r0, vo, 16 * (q >> 1) * PL::T);
      w1 = ld4(r1, vo, 16 * (q >> 1) * PL::T);
    }
    const cf h0 = (q & 1) ? mk(w0.z, w0.w) : mk(w0.x, w0.y);
    const cf h1 = (q & 1) ? mk(w1.z, w1.w) : mk(w1.x, w1.y);
    if (q == SP) {
      const cf c0 = cmac(Y0[q], h0, X[q]), c1 = cmac(Y1[q], h1, X[q]);
      const cf d0 = mk(__builtin_fmaf(h0.x, X[q].x, Y0[q].x), __builtin_fmaf(h0.y, X[q].y, Y0[q].y));
      const cf d1 = mk(__builtin_fmaf(h1.x, X[q].x, Y1[q].x), __builtin_fmaf(h1.y, X[q].y, Y1[q].y));
      Y0[q] = t == 0 ? d0 : c0;
      Y1[q] = t == 0 ? d1 : c1;
    } else {
      Y0[q] = cmac(Y0[q], h0, X[q]);
      Y1[q] = cmac(Y1[q], h1, X[q]);
    }
  }
}

// Inverse-transform one mic spectrum and overlap-add it into y: positions
// m < lim are written; positions m < carry already hold the tails of earlier
// blocks (written by this workgroup) and are accumulated.  Both limits are
// buffer range checks, so no element needs a branch.
template <class PL, class XC>
__device__ __forceinline__ void emit(cf* Yv, XC& lds, const TwBase& tw, float* __restrict__ yp, int lim,
                                     int carry, int t_) {
  Fft<PL>::pre(Yv, tw, t_);
  Fft<PL>::inverse(Yv, lds, tw, t_);
  const int t = opaque_v(t_);
  const rsrc_t wr = make_rsrc(yp, lim * 4);
  const rsrc_t rd = make_rsrc(yp, min(carry, lim) * 4);
  const int vo = 8 * t;
  // Every carry word is requested before the first store.  Reads and writes
  // through different resources cannot be told apart by the compiler, so a
  // read placed after a store waits for it: interleaved, the block would
  // cost one memory round trip per slot.
  cf c[PL::P];
#pragma unroll
  for (int r = 0; r < PL::P; ++r) c[r] = ld2(rd, vo + 8 * r * PL::T);
#pragma unroll
  for (int r = 0; r < PL::P; ++r) {
    const int o = vo + 8 * r * PL::T;
    st2(wr, o, mk(Yv[r].x + c[r].x, Yv[r].y + c[r].y));
  }
}

// The overlap-add carry of one mic block, for carries that fit the first CR
// slots (carry <= 2 T CR): c[r] = y at the thread's samples 2(t + rT),
// 2(t + rT) + 1 below min(carry, lim), zero elsewhere.
template <class PL, int CR>
__device__ __forceinline__ void load_carry(cf* c, const float* __restrict__ yp, int lim, int carry, int t_) {
  const int t = opaque_v(t_);
  const rsrc_t rd = make_rsrc(yp, min(carry, lim) * 4);
  const int vo = 8 * t;
#pragma unroll
  for (int r = 0; r < CR; ++r) {
    const int o = vo + 8 * r * PL::T;
    c[r] = ld2(rd, o);
  }
}

// Inverse-transform one mic spectrum, add the preloaded carry (first CR
// slots) and store the samples below lim.
template <class PL, int CR, class XC>
__device__ __forceinline__ void emit_carried(cf* Yv, const cf* c, XC& lds, const TwBase& tw, float* __restrict__ yp,
                                             int lim, int t_) {
  Fft<PL>::pre(Yv, tw, t_);
  Fft<PL>::inverse(Yv, lds, tw, t_);
  const int t = opaque_v(t_);
  const rsrc_t wr = make_rsrc(yp, lim * 4);
  const int vo = 8 * t;
#pragma unroll
  for (int r = 0; r < PL::P; ++r) {
    const int o = vo + 8 * r * PL::T;
    const cf cr = r < CR ? c[r] : mk(0.f, 0.f);
    st2(wr, o, mk(Yv[r].x + cr.x, Yv[r].y + cr.y));
  }
}

// Inverse-transform the first block of a part p > 0 and split its samples:
// those below h (the head, which the previous part's last block also covers
// with its tail) go to the seam buffer sp, those from h up to lim to y.
// Offsets past a resource's range drop the store, so the split needs no
// branch: a pair straddling h stores its second word alone.
template <class PL, class XC>
__device__ __forceinline__ void emit_seam(cf* Yv, XC& lds, const TwBase& tw, float* __restrict__ yp,
                                          float* __restrict__ sp, int lim, int h, int t_) {
  Fft<PL>::pre(Yv, tw, t_);
  Fft<PL>::inverse(Yv, lds, tw, t_);
  const int t = opaque_v(t_);
  const rsrc_t wy = make_rsrc(yp, lim * 4);
  const rsrc_t wsm = make_rsrc(sp, min(h, lim) * 4);
  constexpr int kDrop = 0x7ffffff0;  // beyond any resource's range
#pragma unroll
  for (int r = 0; r < PL::P; ++r) {
    const int n0 = 2 * (t + r * PL::T);
    const int o = 4 * n0;
    st2(wsm, o, Yv[r]);
    st2(wy, n0 >= h ? o : kDrop, Yv[r]);
    st1(wy, n0 + 1 == h ? o + 4 : kDrop, Yv[r].y);
  }
}

// Parts of an utterance under the block split: at most psplit, at most one
// per block, and one when a block's head could reach back past the previous
// block (a forced hop below L - 1), where the overlap spans several blocks.
__device__ __forceinline__ int mix_parts(int psplit, const Sched& S) {
  if (psplit <= 1 || S.hop < S.lmax - 1) return 1;
  return psplit < S.nb ? psplit : S.nb;
}

template <class PL>
__device__ __forceinline__ const cf* plan_tw() {
  return g_tw + tw_off<ilog2c(PL::N)>();
}

// ------------------------------------------------ front end fused into the mix
// The front end of Sec. 3 (the features of rsim_logmel) computed by the mix
// kernel itself, so that the mixed samples never leave the workgroup.  Mics
// per work item it keeps a frame history for, at most.
constexpr int kFeatMics = 8;

// LDS of the fused front end, carved out of the mix kernel's exchange area
// (idle between the mix's transforms): the stage (the kMelWin final samples
// before the block, then the block's final samples) and one exchange buffer
// per 32-thread frame group.
template <class PL>
struct FeatLds {
  using FP = PlanOf<9>;
  static constexpr int kGroups = PL::T / 32;
  static constexpr int kStageCf = (kMelWin + PL::N) / 2;
  static constexpr int kCf = kStageCf + kGroups * XchWave<FP>::kEntries;
};

// One mic's block after its inverse transform (Yv: the block's contribution
// z to y from its base, samples 2(t + rT) and 2(t + rT) + 1).  Adds the
// earlier blocks' overlap sum (acc_rd, lmax - 1 samples) as the unfused
// kernel adds the carry it reads back from y, keeps the new sum past the hop
// in acc_wr for the next block, and turns every frame whose samples are all
// final into its 128 log-Mel features, with the operations of rsim_logmel's
// kernel (a 512-point plan per group of 32 threads, exchanges synchronised
// within the group's wave).  hist holds the kMelWin final samples before the
// block.  Every thread of the workgroup calls it (it contains barriers).
template <class PL>
__device__ __forceinline__ void feat_block(const MixArgs& A, cf* Yv, cf* lds_raw, float* hist, const float* acc_rd,
                                           float* acc_wr, int j, int bk, int nb, int B, int lmax, int lim,
                                           long long fo, int cap, bool ok, int t_) {
  using FP = PlanOf<9>;
  using FL = FeatLds<PL>;
  constexpr int T = PL::T, P = PL::P;
  static_assert(FL::kCf <= max_lds_with_threads<T>(), "the stage and frame buffers fit the exchange area");
  static_assert(XchWave<FP>::kEntries * 2 >= kMelBins + kMelCapMax, "the power spectrum fits a frame buffer");
  const int t = opaque_v(t_);
  constexpr int kDrop = 0x7ffffff0;  // beyond any resource's range
  const rsrc_t rd = make_rsrc(acc_rd, (bk == 0 ? 0 : lmax - 1) * 4);
  const rsrc_t wr = make_rsrc(acc_wr, (lmax - 1) * 4);
  // Every accumulator word is requested before the first store (a read
  // after a store through another resource would wait for it).
  cf c[P];
#pragma unroll
  for (int r = 0; r < P; ++r) c[r] = ld2(rd, 8 * (t + r * T));
#pragma unroll
  for (int r = 0; r < P; ++r) {
    const int n0 = 2 * (t + r * T);
    Yv[r] = mk(Yv[r].x + c[r].x, Yv[r].y + c[r].y);
    st2(wr, n0 >= B ? 4 * (n0 - B) : kDrop, Yv[r]);
    st1(wr, n0 + 1 == B ? 0 : kDrop, Yv[r].y);
  }
  if (!ok) return;  // uniform
  const int cnt = bk == nb - 1 ? lim : B;  // final samples of this block
  float* stage = reinterpret_cast<float*>(lds_raw);
  __syncthreads();  // the inverse transform's exchange reads are done
  for (int k = t; k < kMelWin; k += T) stage[k] = hist[k];
#pragma unroll
  for (int r = 0; r < P; ++r) {
    const int n0 = 2 * (t + r * T);
    if (n0 < cnt) stage[kMelWin + n0] = Yv[r].x;
    if (n0 + 1 < cnt) stage[kMelWin + n0 + 1] = Yv[r].y;
  }
  __syncthreads();
  const int base = bk * B;
  const int f_lo = mel_frames(base), f_hi = mel_frames(base + cnt);
  const int g = t >> 5, l = t & 31;
  XchWave<FP> xw{reinterpret_cast<cf*>(lds_raw) + FL::kStageCf + g * XchWave<FP>::kEntries};
  float* pw = reinterpret_cast<float*>(xw.base);
  if (f_lo + g < f_hi) {
    const TwBase tw9 = Fft<FP>::bases(plan_tw<FP>(), l);
    float w0[kMelCap0], w1[kMelCap1], w2[kMelCap2], w3[kMelCap3];
    int first[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) first[k] = g_mel_first[l + 32 * k];
#pragma unroll
    for (int i = 0; i < kMelCap0; ++i) w0[i] = g_mel_w[(l + 0) * kMelCapMax + i];
#pragma unroll
    for (int i = 0; i < kMelCap1; ++i) w1[i] = g_mel_w[(l + 32) * kMelCapMax + i];
#pragma unroll
    for (int i = 0; i < kMelCap2; ++i) w2[i] = g_mel_w[(l + 64) * kMelCapMax + i];
#pragma unroll
    for (int i = 0; i < kMelCap3; ++i) w3[i] = g_mel_w[(l + 96) * kMelCapMax + i];
    for (int f = f_lo + g; f < f_hi; f += FL::kGroups) {
      // the frame's first sample in the stage
      const int s0 = kMelHop * f - base + kMelWin;
      cf v[FP::P];
#pragma unroll
      for (int r = 0; r < FP::P; ++r) {
        const int k = 2 * (l + r * FP::T);
        v[r] = mk(stage[s0 + k] * g_hann[k], stage[s0 + k + 1] * g_hann[k + 1]);
      }
      Fft<FP>::forward(v, xw, tw9, l);
      Fft<FP>::post(v, tw9, l);  // 2 X
      xw.sync();  // the transform's exchange reads are done before pw overwrites the buffer
#pragma unroll
      for (int q = 0; q < FP::P; ++q) {
        if (l == 0 && q == Fft<FP>::SP) {
          pw[0] = 0.25f * v[q].x * v[q].x;
          pw[FP::M] = 0.25f * v[q].y * v[q].y;
        } else {
          pw[slot_bin<FP>(q, l)] = 0.25f * (v[q].x * v[q].x + v[q].y * v[q].y);
        }
      }
      xw.sync();
      float* out = A.feat + fo + ((long long)j * cap + f) * kMelBands;
      const float m0 = mel_band<kMelCap0>(w0, pw, first[0]);
      const float m1 = mel_band<kMelCap1>(w1, pw, first[1]);
      const float m2 = mel_band<kMelCap2>(w2, pw, first[2]);
      const float m3 = mel_band<kMelCap3>(w3, pw, first[3]);
      out[l] = logf(m0 + 1e-6f);
      out[l + 32] = logf(m1 + 1e-6f);
      out[l + 64] = logf(m2 + 1e-6f);
      out[l + 96] = logf(m3 + 1e-6f);
      xw.sync();  // the band sums have read pw before the next frame's transform writes the buffer
    }
  }
  __syncthreads();  // every frame has read the stage
  for (int k = t; k < kMelWin; k += T) hist[k] = stage[cnt + k];
  __syncthreads();  // before the exchange area serves the next transform
}

// An utterance's source and RIR descriptors, copied into LDS once per work
// item: reading them later costs an LDS access instead of a scalar memory
// round trip at the start of every source item.  Batches with more slots
// than fit read the descriptor arrays directly.
constexpr int kDescMax = 64;
struct DescCache {
  long long src_off[kDescMax];
  long long rir_off[kDescMax];
  int rir_len[kDescMax];
};

struct UttDesc {
  const BatchDev& b;
  const DescCache& c;
  long long s0, r0;  // first source / RIR slot of the utterance
  bool fast_src, fast_rir;
  __device__ long long src_off(int i) const {
    if (fast_src) return uni64(c.src_off[i]);
    return uni64(b.src_off[s0 + i]);
  }
  __device__ long long rir_off(int k) const {
    if (fast_rir) return uni64(c.rir_off[k]);
    return uni64(b.rir_off[r0 + k]);
  }
  __device__ int rir_len(int k) const {
    if (fast_rir) return uni(c.rir_len[k]);
    return uni(b.rir_len[r0 + k]);
  }
};

// Fills the cache for utterance u (I sources); contains a barrier.
__device__ __forceinline__ UttDesc load_desc(const BatchDev& b, DescCache& c, int u, int I, int t, int nthreads) {
  const long long s0 = (long long)u * b.S, r0 = s0 * b.J;
  const bool fs = b.S <= kDescMax, fr = (long long)b.S * b.J <= kDescMax;
  if (fs)
    for (int i = t; i < I; i += nthreads) c.src_off[i] = b.src_off[s0 + i];
  if (fr)
    for (int k = t; k < I * b.J; k += nthreads) {
      c.rir_off[k] = b.rir_off[r0 + k];
      c.rir_len[k] = b.rir_len[r0 + k];
    }
  __syncthreads();
  return UttDesc{b, c, s0, r0, fs, fr};
}

// The spectrum of one RIR block v (its taps, zero-padded) scaled by a, into
// dst in the paired layout.
template <class PL, class XC>
__device__ __forceinline__ void rir_spectrum_store(cf* v, float a, cf* dst, XC& lds, const TwBase& tw, int t) {
  Fft<PL>::forward(v, lds, tw, t);
  Fft<PL>::post(v, tw, t);
#pragma unroll
  for (int q = 0; q < PL::P; ++q) v[q] = mk(v[q].x * a, v[q].y * a);
  store_spec_pair<PL>(dst, v, t);
}

// The RIR spectra of one utterance, once, scaled by alpha / (8M) (which also
// carries the normalisation of the inverse transform); the next RIR is
// requested while the current one is transformed.
template <class PL, class XC>
__device__ __forceinline__ void rir_spectra(const MixArgs& A, const UttDesc& D, int u, int I, int jlo, int jhi,
                                            cf* Hs, XC& lds, const TwBase& tw, int t) {
  constexpr int P = PL::P, M = PL::M;
  const BatchDev& b = A.b;
  const int J = b.J, NS = b.S, JN = jhi - jlo;
  const float cscale = 1.0f / (8.0f * (float)M);
  const int n_rir = I * JN;
  // item k is RIR (i, j) = (k / JN, jlo + k % JN), slot r0 + i J + j
  const long long r0 = (long long)u * NS * J;
  auto slot_of = [&](int k) __attribute__((always_inline)) { return (k / JN) * J + jlo + k % JN; };
  cf vn[P];
  if (n_rir > 0) {
    const int k0 = slot_of(0);
    load_real<PL>(vn, A.h + D.rir_off(k0), D.rir_len(k0), t);
  }
  for (int k = 0; k < n_rir; ++k) {
    cf v[P];
#pragma unroll
    for (int q = 0; q < P; ++q) v[q] = vn[q];
    if (k + 1 < n_rir) {
      const int kn = slot_of(k + 1);
      load_real<PL>(vn, A.h + D.rir_off(kn), D.rir_len(kn), t);
    }
    const int sl = slot_of(k);
    rir_spectrum_store<PL>(v, A.alpha[r0 + sl] * cscale, Hs + (long long)sl * M, lds, tw, t);
  }
}

// One utterance: RIR spectra, then the blocks.  Mics are processed in groups
// of JG (1 or 2) accumulators; when J > JG the source spectra of the current
// block are kept in the workgroup's scratch for the later mic groups.
template <class PL, int JG, int MINW, bool FEAT>
__device__ __forceinline__ void mix_utterance(const MixArgs& A, int u, const Sched& S, int gsel, int part,
                                              int nparts, cf* lds_raw, DescCache& dc, cf* slot, float* s_hist,
                                              int t) {
  constexpr int P = PL::P, M = PL::M;
  // The variant sized for four waves per SIMD keeps one exchange buffer, so
  // that two workgroups fit a CU's LDS.
  Xch<PL, (MINW >= 4)> lds{lds_raw, 0};
  const TwBase tw = Fft<PL>::bases(plan_tw<PL>(), t);
  const BatchDev& b = A.b;
  const int I = uni(b.n_src[u]), J = b.J, NS = b.S, Nx = uni(b.src_len[u]);
  const int B = S.hop, nb = S.nb, tu = S.tu, lmax = S.lmax;
  const int span = B + lmax - 1;
  // this work item's blocks [b0, b1); a part p > 0 leaves its first block's
  // head (below lmax - 1, which the previous part's last block covers with
  // its tail) in its seam buffer
  const int b0 = (int)((long long)nb * part / nparts), b1 = (int)((long long)nb * (part + 1) / nparts);
  float* seam = part > 0 ? A.seam + ((long long)u * A.psplit + part) * J * A.mmax : nullptr;
  // the RIR spectra: shared by the block ranges (split), else formed into
  // the slot; the source spectra cached for later mic groups follow them
  // in the slot (at its start when the slot holds no RIR spectra)
  cf* Hs = A.hspec ? A.hspec + (long long)u * NS * J * A.mmax : slot;
  cf* Xs = A.hspec ? slot : slot + (long long)NS * J * M;
  const int ng_all = (J + JG - 1) / JG;
  // mic groups of this work item: all, or the one group gsel; the source
  // spectra are cached for later groups only when one item does several
  const int glo = gsel < 0 ? 0 : gsel, ghi = gsel < 0 ? ng_all : gsel + 1;
  const int ng = ghi - glo;
  const bool cache = ng > 1;

  const UttDesc D = load_desc(b, dc, u, I, t, PL::T);
  if (!A.hspec) rir_spectra<PL>(A, D, u, I, glo * JG, min(J, ghi * JG), Hs, lds, tw, t);

  // The fused front end: its features' place, and per mic two overlap-add
  // accumulators of 2 mmax samples at the end of the workgroup's slot.
  long long fo = 0;
  int cap = 0;
  bool fok = false;
  float* accb = nullptr;
  if constexpr (FEAT) {
    fo = uni64(A.feat_off[u]);
    cap = mel_frames(uni(b.out_stride[u]));
    fok = tu < kMelMaxT && J <= kFeatMics && fo >= 0 && fo + (long long)J * cap * kMelBands <= A.feat_len;
    if (!fok && t == 0 && glo == 0) flag_status(RSIM_DEV_BADDESC);
    accb = reinterpret_cast<float*>(slot + A.slot_cf - 2LL * J * A.mmax);
  }
  auto feat_emit = [&](cf* Yv, int j, int bk, int lim) __attribute__((always_inline)) {
    if constexpr (FEAT) {
      Fft<PL>::pre(Yv, tw, t);
      Fft<PL>::inverse(Yv, lds, tw, t);
      float* a0 = accb + (long long)(2 * j) * 2 * A.mmax;
      feat_block<PL>(A, Yv, lds_raw, s_hist + j * kMelWin, a0 + ((bk & 1) ^ 1) * 2 * A.mmax,
                     a0 + (bk & 1) * 2 * A.mmax, j, bk, nb, B, lmax, lim, fo, cap, fok, t);
    }
  };

  const long long yo = uni64(b.out_off[u]);
  const long long ys = uni(b.out_stride[u]);
  // When the register budget allows (16 points per thread and few enough
  // waves per SIMD), the RIR spectra of a source are requested when its
  // iteration starts and the next source's block while the current one is
  // transformed, so the loads overlap the FFT.  The live set is then about
  // (3 + 2 JG) arrays of P complex values.
  constexpr int kWavesPerSimd = MINW > PL::T / 256 ? MINW : PL::T / 256;
  constexpr bool kPrefetch = P <= 16 && (3 + 2 * JG) * 2 * P <= 512 / kWavesPerSimd;
  if constexpr (kPrefetch) {
    // Work items in order (block, mic group, source).  Xn always holds the
    // input of the next item: the next source of this group, else the first
    // source of the next group (cached spectra), else the first source of
    // the next block, so loads are in flight across group and block ends.
    // The RIR spectra of a source are requested when its item starts.  The
    // live set is about (3 + 2 JG) arrays of P complex values.
    cf Xn[P];
    // The input of item (bk, g, i): source i's block bk for the first group,
    // else its cached spectrum.  Both are element q T + t of the thread's
    // slots, so one load site serves every case (the source and the valid
    // count are chosen first, in scalar registers): the prefetched values
    // then always land in the same registers, and no register copy has to
    // wait for them before they are used.
    auto input_of = [&](int bk, int g, int i, const float*& src, int& nvalid) __attribute__((always_inline)) {
      if (g == glo) {
        const int base = bk * B;
        src = A.x + D.src_off(i) + base;
        nvalid = min(B, Nx - base);
      } else {
        src = reinterpret_cast<const float*>(Xs + (long long)i * M);
        nvalid = 2 * M;
      }
    };
    {
      const float* src;
      int nv;
      input_of(b0, glo, 0, src, nv);
      load_real<PL>(Xn, src, nv, t);
    }
    for (int bk = b0; bk < b1; ++bk) {
      const int base = bk * B;
      const int lim = min(span, tu - base);
      const int carry = bk == b0 ? 0 : lmax - 1;
      for (int g = glo; g < ghi; ++g) {
        const int j0 = g * JG;
        const bool two = JG == 2 && j0 + 1 < J;
        cf Y0[P], Y1[JG == 2 ? P : 1];
#pragma unroll
        for (int q = 0; q < P; ++q) Y0[q] = mk(0.f, 0.f);
        if constexpr (JG == 2) {
#pragma unroll
          for (int q = 0; q < P; ++q) Y1[q] = mk(0.f, 0.f);
        }
        for (int i = 0; i < I; ++i) {
          const cf* H0 = Hs + (long long)(i * J + j0) * M;
          cf X[P], Hp0[P], Hp1[JG == 2 ? P : 1];
          // The prefetched input is taken into X before this item's loads
          // are issued: the wait for it then leaves no later load behind it
          // (the counter of outstanding loads drains in issue order), so the
          // RIR spectra stay in flight through the transform.
#pragma unroll
          for (int q = 0; q < P; ++q) X[q] = opaque_c(Xn[q]);
          asm volatile("" ::: "memory");
          load_spec_pair<PL>(Hp0, H0, t);
          if constexpr (JG == 2) {
            if (two) load_spec_pair<PL>(Hp1, H0 + M, t);
          }
          // With one source, the next group's input is this item's own
          // spectrum, not yet in the cache: it is handed over in registers.
          const bool hand_over = g == glo && I == 1 && cache;
          const float* fsrc = A.x;
          int fn = 0;
          bool fetch = true;
          if (i + 1 < I) input_of(bk, g, i + 1, fsrc, fn);
          else if (g + 1 < ghi && !hand_over) input_of(bk, g + 1, 0, fsrc, fn);
          else if (g + 1 >= ghi && bk + 1 < b1) input_of(bk + 1, glo, 0, fsrc, fn);
          else fetch = false;
          if (fetch) load_real<PL>(Xn, fsrc, fn, t);
          if (g == glo) {
            Fft<PL>::forward(X, lds, tw, t);
            Fft<PL>::post(X, tw, t);
            if (cache) store_spec<PL>(Xs + (long long)i * M, X, t);
            if (hand_over) {
#pragma unroll
              for (int q = 0; q < P; ++q) Xn[q] = X[q];
            }
          }
          mac_regs<PL>(Y0, Hp0, X, t);
          if constexpr (JG == 2) {
            if (two) mac_regs<PL>(Y1, Hp1, X, t);
          }
        }
        // Carries that fit the first P/4 slots of each thread (most RIRs) are
        // requested for both mics before either inverse transform, so their
        // latency is hidden; longer ones are read after the transform, all
        // words of a block before its first store (one round trip).
        float* y0 = A.y + yo + (long long)j0 * ys + base;
        constexpr int CR = P / 4;
        if constexpr (FEAT) {
          feat_emit(Y0, j0, bk, lim);
          if constexpr (JG == 2) {
            if (two) feat_emit(Y1, j0 + 1, bk, lim);
          }
        } else if (seam && bk == b0) {
          float* s0 = seam + (long long)j0 * A.mmax;
          emit_seam<PL>(Y0, lds, tw, y0, s0, lim, lmax - 1, t);
          if constexpr (JG == 2) {
            if (two) emit_seam<PL>(Y1, lds, tw, y0 + ys, s0 + A.mmax, lim, lmax - 1, t);
          }
        } else if (carry <= 2 * PL::T * CR) {
          cf C0[CR], C1[CR];
          load_carry<PL, CR>(C0, y0, lim, carry, t);
          if constexpr (JG == 2) {
            if (two) load_carry<PL, CR>(C1, y0 + ys, lim, carry, t);
          }
          emit_carried<PL, CR>(Y0, C0, lds, tw, y0, lim, t);
          if constexpr (JG == 2) {
            if (two) emit_carried<PL, CR>(Y1, C1, lds, tw, y0 + ys, lim, t);
          }
        } else {
          emit<PL>(Y0, lds, tw, y0, lim, carry, t);
          if constexpr (JG == 2) {
            if (two) emit<PL>(Y1, lds, tw, y0 + ys, lim, carry, t);
          }
        }
      }
    }
  } else {
    static_assert(!FEAT, "the fused front end runs on the prefetching path");
    for (int bk = b0; bk < b1; ++bk) {
      const int base = bk * B;
      const int nvalid = min(B, Nx - base);
      const int lim = min(span, tu - base);
      const int carry = bk == b0 ? 0 : lmax - 1;
      for (int g = glo; g < ghi; ++g) {
        const int j0 = g * JG;
        const bool two = JG == 2 && j0 + 1 < J;
        cf Y0[P], Y1[JG == 2 ? P : 1];
#pragma unroll
        for (int q = 0; q < P; ++q) Y0[q] = mk(0.f, 0.f);
        if constexpr (JG == 2) {
#pragma unroll
          for (int q = 0; q < P; ++q) Y1[q] = mk(0.f, 0.f);
        }
        for (int i = 0; i < I; ++i) {
          cf X[P];
          const cf* H0 = Hs + (long long)(i * J + j0) * M;
          if (g == glo) {
            load_real<PL>(X, A.x + D.src_off(i) + base, nvalid, t);
            Fft<PL>::forward(X, lds, tw, t);
            Fft<PL>::post(X, tw, t);
            if (cache) store_spec<PL>(Xs + (long long)i * M, X, t);
          } else {
            load_spec<PL>(X, Xs + (long long)i * M, t);
          }
          if constexpr (JG == 2) {
            if (two) mac2<PL>(Y0, Y1, H0, H0 + M, X, t);
            else mac<PL>(Y0, H0, X, t);
          } else {
            mac<PL>(Y0, H0, X, t);
          }
        }
        if (seam && bk == b0) {
          float* s0 = seam + (long long)j0 * A.mmax;
          emit_seam<PL>(Y0, lds, tw, A.y + yo + (long long)j0 * ys + base, s0, lim, lmax - 1, t);
          if constexpr (JG == 2) {
            if (two)
              emit_seam<PL>(Y1, lds, tw, A.y + yo + (long long)(j0 + 1) * ys + base, s0 + A.mmax, lim, lmax - 1, t);
          }
        } else {
          emit<PL>(Y0, lds, tw, A.y + yo + (long long)j0 * ys + base, lim, carry, t);
          if constexpr (JG == 2) {
            if (two) emit<PL>(Y1, lds, tw, A.y + yo + (long long)(j0 + 1) * ys + base, lim, carry, t);
          }
        }
      }
    }
  }
}

// Persistent workgroups: pop the next utterance of this family's list until
// it is exhausted.  MINW is the number of waves per SIMD the register budget
// is sized for (2 with one mic accumulator, 1 with two).
template <int T, int JG, int MINW, bool FEAT = false>
__global__ __launch_bounds__(T, MINW) void mix_kernel(MixArgs A) {
  __shared__ cf lds[MINW >= 4 ? max_lds_single_with_threads<T>() : max_lds_with_threads<T>()];
  __shared__ DescCache s_desc;
  __shared__ int s_idx;
  __shared__ float s_hist[FEAT ? kFeatMics * kMelWin : 1];
  const int t = threadIdx.x;
  cf* slot = A.scratch + (long long)blockIdx.x * A.slot_cf;
  // The first item of workgroup b is item b; later ones are popped from the
  // family's counter (offset by the grid), so an empty family costs one load
  // per workgroup and no atomic.
  const int gs = A.gsplit, ps = A.psplit, per = gs * ps;
  const int count = __builtin_amdgcn_readfirstlane(A.hdr->count[A.fam]) * per;
  for (int first = 1;; first = 0) {
    __syncthreads();
    if (t == 0) s_idx = first ? (int)blockIdx.x : (int)gridDim.x + atomicAdd(&A.hdr->counter[A.fam], 1);
    __syncthreads();
    // Work-item values are uniform across the workgroup; saying so keeps the
    // descriptor loads scalar and the buffer resources in scalar registers.
    const int idx = __builtin_amdgcn_readfirstlane(s_idx);
    if (idx >= count) break;
    const int pos = idx / per, rem = idx - pos * per;
    const int gsel = gs > 1 ? rem / ps : -1, part = rem % ps;
    const int u = __builtin_amdgcn_readfirstlane(A.list[(long long)A.fam * A.b.U + pos]);
    Sched S = A.sched[u];
    S.log2n = __builtin_amdgcn_readfirstlane(S.log2n);
    S.hop = __builtin_amdgcn_readfirstlane(S.hop);
    S.nb = __builtin_amdgcn_readfirstlane(S.nb);
    S.tu = __builtin_amdgcn_readfirstlane(S.tu);
    S.lmax = __builtin_amdgcn_readfirstlane(S.lmax);
    const int nparts = mix_parts(ps, S);
    if (part >= nparts) continue;
    dispatch_plan<T>(S.log2n, [&](auto pl) __attribute__((always_inline)) {
      using PL = decltype(pl);
      // a group past the utterance's mics has no work
      if (gsel * JG < A.b.J) mix_utterance<PL, JG, MINW, FEAT>(A, u, S, gsel, part, nparts, lds, s_desc, slot, s_hist, t);
    });
  }
}

// First pass of a block-split mix: the spectrum of every RIR slot of the
// family's utterances, scaled by alpha / (8M), into A.hspec (one work item
// per slot), the same operations as the unsplit kernel's, so the parts share
// bit-identical spectra.
template <int T>
__global__ __launch_bounds__(T, 2) void mix_rir_kernel(MixArgs A) {
  __shared__ cf lds_raw[max_lds_with_threads<T>()];
  const int t = threadIdx.x;
  const BatchDev& b = A.b;
  const int NS = b.S, J = b.J;
  const long long per = (long long)NS * J;
  const long long items = (long long)__builtin_amdgcn_readfirstlane(A.hdr->count[A.fam]) * per;
  for (long long k = blockIdx.x; k < items; k += gridDim.x) {
    const int pos = (int)(k / per), i = (int)((k % per) / J), j = (int)(k % J);
    const int u = __builtin_amdgcn_readfirstlane(A.list[(long long)A.fam * b.U + pos]);
    const int log2n = __builtin_amdgcn_readfirstlane(A.sched[u].log2n);
    if (i >= uni(b.n_src[u])) continue;
    const long long r = ((long long)u * NS + i) * J + j;
    // The previous item's transform ended with reads of the exchange buffer
    // this item's first exchange writes (its parity starts again at 0).
    __syncthreads();
    dispatch_plan<T>(log2n, [&](auto pl) __attribute__((always_inline)) {
      using PL = decltype(pl);
      Xch<PL> lds{lds_raw, 0};
      const TwBase tw = Fft<PL>::bases(plan_tw<PL>(), t);
      cf v[PL::P];
      load_real<PL>(v, A.h + uni64(b.rir_off[r]), uni(b.rir_len[r]), t);
      const float cscale = 1.0f / (8.0f * (float)PL::M);
      rir_spectrum_store<PL>(v, A.alpha[r] * cscale, A.hspec + (long long)u * per * A.mmax + (long long)(i * J + j) * PL::M,
                             lds, tw, t);
    });
  }
}

// Last pass of a block-split mix: for every part p > 0 of an utterance and
// every mic, the head its first block left in the seam buffer is added to
// the tail the previous part's last block stored in y.  The two operands are
// the ones the unsplit kernel adds (in the other order; the sum is the same),
// so the outputs are bit-identical to the unsplit kernel's.
// Each thread requests kSeamPer elements of both operands before it adds
// and stores any (the seam buffer and y never overlap), so a seam of up to
// kSeamThreads * kSeamPer samples costs one memory round trip.
constexpr int kSeamThreads = 256, kSeamPer = 16;
__global__ __launch_bounds__(kSeamThreads) void mix_seam_kernel(MixArgs A) {
  const BatchDev& b = A.b;
  const int J = b.J, ps = A.psplit;
  const long long per = (long long)ps * J;
  const long long items = (long long)A.hdr->count[A.fam] * per;
  for (long long k = blockIdx.x; k < items; k += gridDim.x) {
    const int pos = (int)(k / per), part = (int)((k % per) / J), j = (int)(k % J);
    const int u = A.list[(long long)A.fam * b.U + pos];
    const Sched S = A.sched[u];
    const int nparts = mix_parts(ps, S);
    if (part == 0 || part >= nparts) continue;
    const int b0 = (int)((long long)S.nb * part / nparts);
    const int base = b0 * S.hop;
    const int h = min(S.lmax - 1, S.tu - base);
    float* __restrict__ y = A.y + b.out_off[u] + (long long)j * b.out_stride[u] + base;
    const float* __restrict__ sm = A.seam + (((long long)u * ps + part) * J + j) * A.mmax;
    for (int n0 = 0; n0 < h; n0 += kSeamThreads * kSeamPer) {
      float yv[kSeamPer], sv[kSeamPer];
#pragma unroll
      for (int e = 0; e < kSeamPer; ++e) {
        const int n = n0 + e * kSeamThreads + (int)threadIdx.x;
        yv[e] = n < h ? y[n] : 0.0f;
        sv[e] = n < h ? sm[n] : 0.0f;
      }
#pragma unroll
      for (int e = 0; e < kSeamPer; ++e) {
        const int n = n0 + e * kSeamThreads + (int)threadIdx.x;
        if (n < h) y[n] = yv[e] + sv[e];
      }
    }
  }
}

// ============================================================== the adjoint
// Y += conj(A) B over the thread's slots, A and B from memory (slot SP of
// thread 0 holds two real bins, for which conj is the identity).
template <class PL>
__device__ __forceinline__ void macc_mem(cf* Y, const cf* __restrict__ Am, const cf* __restrict__ Bm, int t_) {
  constexpr int SP = Fft<PL>::SP;
  const int t = opaque_v(t_);
  const rsrc_t ra = make_rsrc(Am, PL::P * PL::T * 8);
  const rsrc_t rb = make_rsrc(Bm, PL::P * PL::T * 8);
  const int vo = 16 * t;  // paired layout: slot q at (q / 2) 2T + 2t + q % 2
#pragma unroll
  for (int q = 0; q < PL::P; ++q) {
    const cf a = ld2(ra, vo + 8 * (q & 1), 16 * (q >> 1) * PL::T);
    const cf bv = ld2(rb, vo + 8 * (q & 1), 16 * (q >> 1) * PL::T);
    if (q == SP) {
      const cf c = cmacc(Y[q], a, bv);
      const cf d = mk(__builtin_fmaf(a.x, bv.x, Y[q].x), __builtin_fmaf(a.y, bv.y, Y[q].y));
      Y[q] = t == 0 ? d : c;
    } else {
      Y[q] = cmacc(Y[q], a, bv);
    }
  }
}

// R (memory) = (first ? 0 : R) + conj(X) B, X in registers, B from memory.
template <class PL>
__device__ __forceinline__ void acc_corr(cf* __restrict__ Rm, const cf* X, const cf* __restrict__ Bm, bool first,
                                         int t_) {
  constexpr int SP = Fft<PL>::SP;
  const int t = opaque_v(t_);
  const rsrc_t rr = make_rsrc(Rm, first ? 0 : PL::P * PL::T * 8);  // a zero range reads zeros
  const rsrc_t rw = make_rsrc(Rm, PL::P * PL::T * 8);
  const rsrc_t rb = make_rsrc(Bm, PL::P * PL::T * 8);
  const int vo = 16 * t;  // paired layout
  // Slots in batches of QB, all operands of a batch requested before its
  // first store (reads and writes through different resources cannot be
  // told apart by the compiler: a read after a store waits for it).
  constexpr int QB = PL::P < 8 ? PL::P : 8;
#pragma unroll
  for (int q0 = 0; q0 < PL::P; q0 += QB) {
    cf acc[QB], bv[QB];
#pragma unroll
    for (int e = 0; e < QB; ++e) {
      const int q = q0 + e;
      const int vq = vo + 8 * (q & 1), sq = 16 * (q >> 1) * PL::T;
      acc[e] = ld2(rr, vq, sq);
      bv[e] = ld2(rb, vq, sq);
    }
#pragma unroll
    for (int e = 0; e < QB; ++e) {
      const int q = q0 + e;
      const int vq = vo + 8 * (q & 1), sq = 16 * (q >> 1) * PL::T;
      cf o;
      if (q == SP) {
        const cf c = cmacc(acc[e], X[q], bv[e]);
        const cf d = mk(__builtin_fmaf(X[q].x, bv[e].x, acc[e].x), __builtin_fmaf(X[q].y, bv[e].y, acc[e].y));
        o = t == 0 ? d : c;
      } else {
        o = cmacc(acc[e], X[q], bv[e]);
      }
      st2(rw, vq, o, sq);
    }
  }
}

// One source against every mic for two blocks b, b + 1 (the second may be
// absent: g1 then has a zero range and reads zeros, and X1 is zero):
//   D0 += conj(H_ij) G_j,b,   D1 += conj(H_ij) G_j,b+1          (registers)
//   R_ij = (first ? 0 : R_ij) + conj(X0) G_j,b + conj(X1) G_j,b+1   (memory)
// so each RIR spectrum, gradient spectrum and accumulator is read once per
// pair of blocks.  H_ij, G_j,b, G_j,b+1 and R_ij are spectra M apart.
template <class PL>
__device__ __forceinline__ void bwd_pair_pass(cf* D0, cf* D1, const cf* X0, const cf* X1,
                                              const cf* __restrict__ Hi, const cf* __restrict__ G0,
                                              const cf* __restrict__ G1, cf* __restrict__ Ri, int J, bool first,
                                              bool two, int t_) {
  constexpr int SP = Fft<PL>::SP, M = PL::M;
  // Slots in batches of QB: all operands of a batch are requested before any
  // of its accumulators is written back (the compiler cannot tell the
  // accumulator reads from the writes apart, so reads after a write wait for
  // it), which makes one memory round trip per batch instead of per slot.
  // The spectra are in the paired layout: one 128-bit access per two slots.
  constexpr int QB = PL::P < 8 ? PL::P : 8;
  const int t = opaque_v(t_);
  const int vo = 16 * t;
  constexpr int bytes = PL::P * PL::T * 8;
  typedef unsigned u4 __attribute__((ext_vector_type(4)));
  for (int j = 0; j < J; ++j) {
    const rsrc_t rh = make_rsrc(Hi + (long long)j * M, bytes);
    const rsrc_t r0 = make_rsrc(G0 + (long long)j * M, bytes);
    const rsrc_t r1 = make_rsrc(G1 + (long long)j * M, two ? bytes : 0);
    const rsrc_t rr = make_rsrc(Ri + (long long)j * M, first ? 0 : bytes);
    const rsrc_t rw = make_rsrc(Ri + (long long)j * M, bytes);
#pragma unroll
    for (int q0 = 0; q0 < PL::P; q0 += QB) {
      f4 hb[QB / 2], g0b[QB / 2], g1b[QB / 2], ab[QB / 2];
#pragma unroll
      for (int e = 0; e < QB / 2; ++e) {
        const int so = 16 * (q0 / 2 + e) * PL::T;
        hb[e] = ld4(rh, vo, so);
        g0b[e] = ld4(r0, vo, so);
        g1b[e] = ld4(r1, vo, so);
        ab[e] = ld4(rr, vo, so);
      }
#pragma unroll
      for (int e = 0; e < QB / 2; ++e) {
        cf o2[2];
#pragma unroll
        for (int hlf = 0; hlf < 2; ++hlf) {
          const int q = q0 + 2 * e + hlf;
          const cf h = hlf ? mk(hb[e].z, hb[e].w) : mk(hb[e].x, hb[e].y);
          const cf g0 = hlf ? mk(g0b[e].z, g0b[e].w) : mk(g0b[e].x, g0b[e].y);
          const cf g1 = hlf ? mk(g1b[e].z, g1b[e].w) : mk(g1b[e].x, g1b[e].y);
          const cf acc = hlf ? mk(ab[e].z, ab[e].w) : mk(ab[e].x, ab[e].y);
          cf o;
          if (q == SP) {
            const cf c0 = cmacc(D0[q], h, g0), c1 = cmacc(D1[q], h, g1);
            const cf co = cmacc(cmacc(acc, X0[q], g0), X1[q], g1);
            const cf d0 = mk(__builtin_fmaf(h.x, g0.x, D0[q].x), __builtin_fmaf(h.y, g0.y, D0[q].y));
            const cf d1 = mk(__builtin_fmaf(h.x, g1.x, D1[q].x), __builtin_fmaf(h.y, g1.y, D1[q].y));
            const cf dr = mk(__builtin_fmaf(X1[q].x, g1.x, __builtin_fmaf(X0[q].x, g0.x, acc.x)),
                             __builtin_fmaf(X1[q].y, g1.y, __builtin_fmaf(X0[q].y, g0.y, acc.y)));
            D0[q] = t == 0 ? d0 : c0;
            D1[q] = t == 0 ? d1 : c1;
            o = t == 0 ? dr : co;
          } else {
            D0[q] = cmacc(D0[q], h, g0);
            D1[q] = cmacc(D1[q], h, g1);
            o = cmacc(cmacc(acc, X0[q], g0), X1[q], g1);
          }
          o2[hlf] = o;
        }
        const f4 w = {o2[0].x, o2[0].y, o2[1].x, o2[1].y};
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, w), rw, vo, 16 * (q0 / 2 + e) * PL::T, 0);
      }
    }
  }
}

// Inverse-transform a spectrum and store the first `lim` samples at yp.
template <class PL>
__device__ __forceinline__ void emit_store(cf* Yv, Xch<PL>& lds, const TwBase& tw, float* __restrict__ yp, int lim,
                                           int t_) {
  Fft<PL>::pre(Yv, tw, t_);
  Fft<PL>::inverse(Yv, lds, tw, t_);
  const int t = opaque_v(t_);
  const rsrc_t wr = make_rsrc(yp, lim * 4);
  const int vo = 8 * t;
#pragma unroll
  for (int r = 0; r < PL::P; ++r) {
    const int o = vo + 8 * r * PL::T;
    st2(wr, o, Yv[r]);
  }
}

// Sum over the workgroup's T threads (T a power of two, any T <= 1024): a
// tree in LDS, so partial waves (T = 32) need no cross-lane operation.
template <int T>
__device__ __forceinline__ double block_sum_d(double v, double* s_red, int t) {
  __syncthreads();  // earlier readers of s_red are done
  s_red[t] = v;
  __syncthreads();
#pragma unroll
  for (int h = T / 2; h > 0; h >>= 1) {
    if (t < h) s_red[t] += s_red[t + h];
    __syncthreads();
  }
  return s_red[0];
}

// One utterance of the adjoint.  With g_j the output gradient of mic j:
//   dx_i[n]   = sum_j alpha_ij (h_ij corr g_j)[n]        per block, overlap-save
//   r_ij[k]   = sum_n x_i[n] g_j[n + k]                  spectra summed over blocks
//   dh_ij[k]  = alpha_ij r_ij[k],   dalpha_ij = sum_k h_ij[k] r_ij[k]
// Block b of the output gradient, g_j[bB .. bB + N), holds every sample the
// block's dx and the block's share of r need (B + L_max - 1 <= N, no wrap).
// Scratch: alpha-scaled RIR spectra (I J), this block's gradient spectra (J)
// and the correlation accumulators (I J).
// r_ij from its spectrum (sum of `nparts` accumulators `stride` entries
// apart): dh = alpha r below L (zero from L to L0), dalpha = <h, r> in FP64.
template <class PL>
__device__ __forceinline__ void bwd_finish_rir(const BwdArgs& A, long long r, const cf* R, int nparts,
                                               long long stride, Xch<PL>& lds, const TwBase& tw, double* s_red,
                                               int t) {
  constexpr int P = PL::P;
  const BatchDev& b = A.b;
  const int L = uni(b.rir_len[r]), L0 = uni(b.rir_len0[r]);
  const long long ro = uni64(b.rir_off[r]);
  const float a = A.alpha[r];
  // With 1024 threads (128 registers each) the parts and taps are read as
  // they are needed; otherwise every part is requested at once (then summed
  // in part order) and the kept taps before the transform.
  constexpr bool kBatch = PL::T <= 512;
  cf v[P];
  load_spec_pair<PL>(v, R, t);
  if (kBatch && nparts <= 4) {
    cf w1[kBatch ? P : 1], w2[kBatch ? P : 1], w3[kBatch ? P : 1];
    if (nparts > 1) load_spec_pair<PL>(w1, R + stride, t);
    if (nparts > 2) load_spec_pair<PL>(w2, R + 2 * stride, t);
    if (nparts > 3) load_spec_pair<PL>(w3, R + 3 * stride, t);
    if (nparts > 1) {
#pragma unroll
      for (int q = 0; q < P; ++q) v[q] = mk(v[q].x + w1[q].x, v[q].y + w1[q].y);
    }
    if (nparts > 2) {
#pragma unroll
      for (int q = 0; q < P; ++q) v[q] = mk(v[q].x + w2[q].x, v[q].y + w2[q].y);
    }
    if (nparts > 3) {
#pragma unroll
      for (int q = 0; q < P; ++q) v[q] = mk(v[q].x + w3[q].x, v[q].y + w3[q].y);
    }
  } else {
    for (int k = 1; k < nparts; ++k) {
      cf w[P];
      load_spec_pair<PL>(w, R + k * stride, t);
#pragma unroll
      for (int q = 0; q < P; ++q) v[q] = mk(v[q].x + w[q].x, v[q].y + w[q].y);
    }
  }
  const rsrc_t hr = make_rsrc(A.h + ro, L * 4);
  cf hv_all[kBatch ? P : 1];
  if constexpr (kBatch) {
#pragma unroll
    for (int q = 0; q < P; ++q) hv_all[q] = ld2(hr, 8 * (t + q * PL::T));
  }
  Fft<PL>::pre(v, tw, t);
  Fft<PL>::inverse(v, lds, tw, t);
  // v[q] holds r at samples 2(t + qT), 2(t + qT) + 1.
  const rsrc_t gw = make_rsrc(A.gh + ro, L * 4);
  double part = 0.0;
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const int o = 8 * (t + q * PL::T);
    cf hv;
    if constexpr (kBatch) hv = hv_all[q];
    else hv = ld2(hr, o);
    part += (double)hv.x * (double)v[q].x + (double)hv.y * (double)v[q].y;
    st2(gw, o, mk(a * v[q].x, a * v[q].y));
  }
  const double da = block_sum_d<PL::T>(part, s_red, t);
  if (t == 0 && A.galpha) A.galpha[r] = (float)da;
  for (int k = L + t; k < L0; k += PL::T) A.gh[ro + k] = 0.0f;
}

// The alpha-scaled spectrum of RIR slot r (its kept taps) into dst.
template <class PL>
__device__ __forceinline__ void bwd_rir_spectrum(const BwdArgs& A, long long r, cf* dst, Xch<PL>& lds,
                                                 const TwBase& tw, int t) {
  constexpr int P = PL::P;
  const BatchDev& b = A.b;
  cf v[P];
  load_real<PL>(v, A.h + uni64(b.rir_off[r]), uni(b.rir_len[r]), t);
  Fft<PL>::forward(v, lds, tw, t);
  Fft<PL>::post(v, tw, t);
  const float a = A.alpha[r];
#pragma unroll
  for (int q = 0; q < P; ++q) v[q] = mk(v[q].x * a, v[q].y * a);
  store_spec_pair<PL>(dst, v, t);
}

// Work item (u, part) of the adjoint: blocks [b0, b1) of utterance u.  With
// one part per utterance it also finishes dh and dalpha; otherwise it leaves
// its correlation spectra in A.partial for the finishing pass.
template <class PL>
__device__ __forceinline__ void bwd_utterance(const BwdArgs& A, int u, const Sched& S, int part, int nparts,
                                              cf* lds_raw, double* s_red, cf* slot, int t) {
  constexpr int P = PL::P, M = PL::M, N = PL::N;
  Xch<PL> lds{lds_raw, 0};
  const TwBase tw = Fft<PL>::bases(plan_tw<PL>(), t);
  const BatchDev& b = A.b;
  const int I = uni(b.n_src[u]), J = b.J, NS = b.S, Nx = uni(b.src_len[u]);
  const int B = S.hop, nb = S.nb, tu = S.tu;
  const float gscale = 1.0f / (8.0f * (float)M);
  cf* Hs = A.hspec ? A.hspec + (long long)u * NS * J * A.mmax : slot;
  cf* Gs = slot + (long long)NS * J * M;
  cf* Rs = nparts == 1 ? Gs + 2LL * J * M
                       : A.partial + ((long long)u * A.nsplit + part) * NS * J * A.mmax;
  const int b0 = (int)((long long)nb * part / nparts), b1 = (int)((long long)nb * (part + 1) / nparts);
  const long long yo = uni64(b.out_off[u]);
  const long long ys = uni(b.out_stride[u]);

  if (!A.hspec) {
    for (int i = 0; i < I; ++i)
      for (int j = 0; j < J; ++j)
        bwd_rir_spectrum<PL>(A, ((long long)u * NS + i) * J + j, Hs + (long long)(i * J + j) * M, lds, tw, t);
  }

  if constexpr (PL::T <= 512) {
    // Two blocks per pass: the gradient spectra of both blocks are stored,
    // then per source both source spectra are formed and one pass over the
    // mics gives both blocks' dx spectra and their share of r.
    for (int bk = b0; bk < b1; bk += 2) {
      const bool two = bk + 1 < b1;
      // the gradient blocks (block hb, mic j) = item k = hb J + j, the next
      // one requested while the current one is transformed
      const int ng = (two ? 2 : 1) * J;
      auto grad_src = [&](int k, const float*& src, int& nv) __attribute__((always_inline)) {
        const int hb = k / J, j = k - hb * J;
        const int base = (bk + hb) * B;
        src = A.gy + yo + (long long)j * ys + base;
        nv = min(N, tu - base);
      };
      cf vn[P];
      {
        const float* src;
        int nv;
        grad_src(0, src, nv);
        load_real<PL>(vn, src, nv, t);
      }
      for (int k = 0; k < ng; ++k) {
        cf v[P];
#pragma unroll
        for (int q = 0; q < P; ++q) v[q] = opaque_c(vn[q]);
        asm volatile("" ::: "memory");
        if (k + 1 < ng) {
          const float* src;
          int nv;
          grad_src(k + 1, src, nv);
          load_real<PL>(vn, src, nv, t);
        }
        Fft<PL>::forward(v, lds, tw, t);
        Fft<PL>::post(v, tw, t);
#pragma unroll
        for (int q = 0; q < P; ++q) v[q] = mk(v[q].x * gscale, v[q].y * gscale);
        store_spec_pair<PL>(Gs + (long long)k * M, v, t);
      }
      for (int i = 0; i < I; ++i) {
        const long long so = uni64(b.src_off[(long long)u * NS + i]);
        const int base0 = bk * B, base1 = base0 + B;
        const int nv0 = min(B, Nx - base0), nv1 = two ? min(B, Nx - base1) : 0;
        cf X0[P], X1[P], D0[P], D1[P];
        // both blocks are requested before the first transform (the second
        // reads zeros when there is no second block)
        load_real<PL>(X0, A.x + so + base0, nv0, t);
        load_real<PL>(X1, A.x + so + base1, nv1, t);
        Fft<PL>::forward(X0, lds, tw, t);
        Fft<PL>::post(X0, tw, t);
        if (two) {
          Fft<PL>::forward(X1, lds, tw, t);
          Fft<PL>::post(X1, tw, t);
        }
#pragma unroll
        for (int q = 0; q < P; ++q) D0[q] = D1[q] = mk(0.f, 0.f);
        bwd_pair_pass<PL>(D0, D1, X0, X1, Hs + (long long)i * J * M, Gs, Gs + (long long)J * M,
                          Rs + (long long)i * J * M, J, bk == b0, two, t);
        emit_store<PL>(D0, lds, tw, A.gx + so + base0, nv0, t);
        if (two) emit_store<PL>(D1, lds, tw, A.gx + so + base1, nv1, t);
      }
    }
  } else {
    for (int bk = b0; bk < b1; ++bk) {
      const int base = bk * B;
      const int nvalid = min(B, Nx - base);
      for (int j = 0; j < J; ++j) {
        cf v[P];
        load_real<PL>(v, A.gy + yo + (long long)j * ys + base, min(N, tu - base), t);
        Fft<PL>::forward(v, lds, tw, t);
        Fft<PL>::post(v, tw, t);
#pragma unroll
        for (int q = 0; q < P; ++q) v[q] = mk(v[q].x * gscale, v[q].y * gscale);
        store_spec_pair<PL>(Gs + (long long)j * M, v, t);
      }
      for (int i = 0; i < I; ++i) {
        const long long so = uni64(b.src_off[(long long)u * NS + i]);
        cf D[P];
#pragma unroll
        for (int q = 0; q < P; ++q) D[q] = mk(0.f, 0.f);
        for (int j = 0; j < J; ++j) macc_mem<PL>(D, Hs + (long long)(i * J + j) * M, Gs + (long long)j * M, t);
        emit_store<PL>(D, lds, tw, A.gx + so + base, nvalid, t);
        cf X[P];
        load_real<PL>(X, A.x + so + base, nvalid, t);
        Fft<PL>::forward(X, lds, tw, t);
        Fft<PL>::post(X, tw, t);
        for (int j = 0; j < J; ++j)
          acc_corr<PL>(Rs + (long long)(i * J + j) * M, X, Gs + (long long)j * M, bk == b0, t);
      }
    }
  }
  if (b1 == b0) {  // an empty part still defines its share: zero
    for (int k = 0; k < I * J; ++k) {
      cf z[P];
#pragma unroll
      for (int q = 0; q < P; ++q) z[q] = mk(0.f, 0.f);
      store_spec_pair<PL>(Rs + (long long)k * M, z, t);
    }
  }
  if (nparts > 1) return;

  for (int i = 0; i < I; ++i)
    for (int j = 0; j < J; ++j)
      bwd_finish_rir<PL>(A, ((long long)u * NS + i) * J + j, Rs + (long long)(i * J + j) * M, 1, 0, lds, tw,
                         s_red, t);
}

// Work item of the adjoint: (list position, part).  nsplit parts per
// utterance, capped by its block count (parts beyond it have no work).
__device__ __forceinline__ int bwd_parts(int nsplit, int nb) { return nsplit < nb ? nsplit : nb; }

template <int T>
__global__ __launch_bounds__(T, 2) void bwd_kernel(BwdArgs A) {
  __shared__ cf lds[max_lds_with_threads<T>()];
  __shared__ double s_red[T];
  __shared__ int s_idx;
  const int t = threadIdx.x;
  cf* slot = A.scratch + (long long)blockIdx.x * A.slot_cf;
  const int ns = A.nsplit;
  const long long count = (long long)__builtin_amdgcn_readfirstlane(A.hdr->count[A.fam]) * ns;
  for (int first = 1;; first = 0) {
    __syncthreads();
    if (t == 0) s_idx = first ? (int)blockIdx.x : (int)gridDim.x + atomicAdd(&A.hdr->counter[A.fam], 1);
    __syncthreads();
    const int idx = __builtin_amdgcn_readfirstlane(s_idx);
    if (idx >= count) break;
    const int pos = idx / ns, part = idx - pos * ns;
    const int u = __builtin_amdgcn_readfirstlane(A.list[(long long)A.fam * A.b.U + pos]);
    Sched S = A.sched[u];
    S.log2n = __builtin_amdgcn_readfirstlane(S.log2n);
    S.hop = __builtin_amdgcn_readfirstlane(S.hop);
    S.nb = __builtin_amdgcn_readfirstlane(S.nb);
    S.tu = __builtin_amdgcn_readfirstlane(S.tu);
    S.lmax = __builtin_amdgcn_readfirstlane(S.lmax);
    const int nparts = bwd_parts(ns, S.nb);
    if (part >= nparts) continue;
    dispatch_plan<T>(S.log2n, [&](auto pl) __attribute__((always_inline)) {
      using PL = decltype(pl);
      bwd_utterance<PL>(A, u, S, part, nparts, lds, s_red, slot, t);
    });
  }
}

// First pass of a split adjoint: the alpha-scaled spectrum of every RIR slot
// of the family's utterances into A.hspec, one work item per slot, so that
// the parts of an utterance share them.
template <int T>
__global__ __launch_bounds__(T, 2) void bwd_rir_kernel(BwdArgs A) {
  __shared__ cf lds_raw[max_lds_with_threads<T>()];
  const int t = threadIdx.x;
  const BatchDev& b = A.b;
  const int NS = b.S, J = b.J;
  const long long per = (long long)NS * J;
  const long long items = (long long)__builtin_amdgcn_readfirstlane(A.hdr->count[A.fam]) * per;
  for (long long k = blockIdx.x; k < items; k += gridDim.x) {
    const int pos = (int)(k / per), i = (int)((k % per) / J), j = (int)(k % J);
    const int u = __builtin_amdgcn_readfirstlane(A.list[(long long)A.fam * b.U + pos]);
    const int log2n = __builtin_amdgcn_readfirstlane(A.sched[u].log2n);
    if (i >= uni(b.n_src[u])) continue;
    // The previous item's transform ended with reads of the exchange buffer
    // this item's first exchange writes (its parity starts again at 0).
    __syncthreads();
    dispatch_plan<T>(log2n, [&](auto pl) __attribute__((always_inline)) {
      using PL = decltype(pl);
      Xch<PL> lds{lds_raw, 0};
      const TwBase tw = Fft<PL>::bases(plan_tw<PL>(), t);
      bwd_rir_spectrum<PL>(A, ((long long)u * NS + i) * J + j,
                           A.hspec + (long long)u * per * A.mmax + (long long)(i * J + j) * PL::M, lds, tw, t);
    });
  }
}

// Finishing pass of a split adjoint: for every RIR slot (i, j) of an
// utterance in more than one part, sums the parts' correlation spectra and
// gives dh and dalpha.  One work item per slot, grid-stride.
template <int T>
__global__ __launch_bounds__(T, 2) void bwd_finish_kernel(BwdArgs A) {
  __shared__ cf lds_raw[max_lds_with_threads<T>()];
  __shared__ double s_red[T];
  const int t = threadIdx.x;
  const BatchDev& b = A.b;
  const int NS = b.S, J = b.J;
  const long long per = (long long)NS * J;
  const long long items = (long long)__builtin_amdgcn_readfirstlane(A.hdr->count[A.fam]) * per;
  for (long long k = blockIdx.x; k < items; k += gridDim.x) {
    const int pos = (int)(k / per), i = (int)((k % per) / J), j = (int)(k % J);
    const int u = __builtin_amdgcn_readfirstlane(A.list[(long long)A.fam * b.U + pos]);
    Sched S = A.sched[u];
    S.log2n = __builtin_amdgcn_readfirstlane(S.log2n);
    S.nb = __builtin_amdgcn_readfirstlane(S.nb);
    const int nparts = bwd_parts(A.nsplit, S.nb);
    if (nparts <= 1 || i >= uni(b.n_src[u])) continue;
    dispatch_plan<T>(S.log2n, [&](auto pl) __attribute__((always_inline)) {
      using PL = decltype(pl);
      constexpr int M = PL::M;
      Xch<PL> lds{lds_raw, 0};
      const TwBase tw = Fft<PL>::bases(plan_tw<PL>(), t);
      const long long stride = per * A.mmax;  // one part's spectra
      const cf* R = A.partial + (long long)u * A.nsplit * stride;
      bwd_finish_rir<PL>(A, ((long long)u * NS + i) * J + j, R + (long long)(i * J + j) * M, nparts, stride,
                         lds, tw, s_red, t);
    });
  }
}

// Utterances without work (no source, no samples or no RIR tap) still get
// their gradients: zeros.  One workgroup per utterance, grid-stride.
__global__ __launch_bounds__(256) void bwd_zero_kernel(BwdArgs A) {
  const BatchDev& b = A.b;
  for (int u = blockIdx.x; u < b.U; u += gridDim.x) {
    const Sched S = A.sched[u];
    if (S.nb > 0) continue;
    const int I = b.n_src[u], J = b.J, NS = b.S, Nx = b.src_len[u];
    if (I < 0 || I > NS || Nx < 0) continue;  // flagged by the schedule
    for (int i = 0; i < I; ++i) {
      const long long so = b.src_off[(long long)u * NS + i];
      if (so < 0 || so + Nx > b.x_len) continue;
      for (int n = threadIdx.x; n < Nx; n += 256) A.gx[so + n] = 0.0f;
      for (int j = 0; j < J; ++j) {
        const long long r = ((long long)u * NS + i) * J + j;
        const long long ro = b.rir_off[r];
        const int L0 = b.rir_len0[r];
        if (L0 < 0 || ro < 0 || ro + L0 > b.h_len) continue;
        for (int k = threadIdx.x; k < L0; k += 256) A.gh[ro + k] = 0.0f;
        if (threadIdx.x == 0 && A.galpha) A.galpha[r] = 0.0f;
      }
    }
  }
}

// ======================================= reverberant energies (gain rule)
// E_ij = sum_n ((h_ij * x_i)[n])^2 for the cut RIRs, from the identity
// E = sum_{|l| < L} r_hh[l] r_xx[l] (r the autocorrelations) evaluated in the
// frequency domain: with N >= 2 Lmax (Lmax the longest kept RIR of source i),
// E_ij = (1/N) sum_k |H_ij[k]|^2 S_i[k], S_i the transform of r_xx
// windowed to |l| < Lmax and made periodic with period N (no aliasing since
// L + Lmax - 1 <= N).  r_xx up to lag Lmax - 1 is accumulated over half
// blocks x_b = x[b N/2, (b + 1) N/2): lag l < Lmax <= N/2 pairs a sample of
// x_b with one of x_b or x_{b+1}, and the window x[b N/2, b N/2 + N) has the
// spectrum X_b + (-1)^k X_{b+1}, so each half block is transformed once and
// r_xx = IFFT(sum_b conj(X_b) (X_b + (-1)^k X_{b+1})) on lags [0, Lmax).
// One work item per source slot.
struct EnergyArgs {
  BatchDev b;
  const float* x;
  const float* h;
  double* energy;  // [U*S*J]
  int fam;
};

// log2 of the transform size for a longest kept RIR of lmax taps: at least
// 2 lmax points, and at least 16384 (long blocks, the most efficient plan).
__host__ __device__ constexpr int energy_log2n(int lmax) {
  int l2 = 14;
  while (l2 < 16 && (1 << l2) < 2 * lmax) ++l2;
  return l2;
}

template <class PL>
__device__ __forceinline__ void energy_source(const EnergyArgs& A, int u, int i, int lmax, cf* lds_raw,
                                              double* s_red, int t) {
#pragma clang fp contract(off)
  constexpr int P = PL::P, M = PL::M, N = PL::N, T = PL::T, SP = Fft<PL>::SP;
  Xch<PL> lds{lds_raw, 0};
  const TwBase tw = Fft<PL>::bases(plan_tw<PL>(), t);
  const BatchDev& b = A.b;
  const int Nx = uni(b.src_len[u]), J = b.J;
  const long long so = uni64(b.src_off[(long long)u * b.S + i]);
  const int nb = (Nx + M - 1) / M;  // half blocks of M = N/2 samples
  // (-1)^k for every bin k this thread holds: its bins have the parity of t
  const float sgn = (t & 1) ? -1.f : 1.f;
  // With 1024 threads (128 registers each) the next half block is not held
  // while the current one is transformed.
  constexpr bool kPrefetch = T <= 512;
  cf R[P], Xc[P], Xn[P];
#pragma unroll
  for (int q = 0; q < P; ++q) R[q] = mk(0.f, 0.f);
  load_real<PL>(Xc, A.x + so, min(M, Nx), t);
  if (kPrefetch && nb > 1) load_real<PL>(Xn, A.x + so + M, min(M, Nx - M), t);
  Fft<PL>::forward(Xc, lds, tw, t);
  Fft<PL>::post(Xc, tw, t);
  for (int bk = 0; bk < nb; ++bk) {
    // X: the spectrum of half block bk + 1 (zero past the end)
    cf X[P];
    if (bk + 1 < nb) {
      const int base = (bk + 1) * M;
      if (!kPrefetch) load_real<PL>(Xn, A.x + so + base, min(M, Nx - base), t);
#pragma unroll
      for (int q = 0; q < P; ++q) X[q] = Xn[q];
      if (kPrefetch && bk + 2 < nb) load_real<PL>(Xn, A.x + so + base + M, min(M, Nx - base - M), t);
      Fft<PL>::forward(X, lds, tw, t);
      Fft<PL>::post(X, tw, t);
    } else {
#pragma unroll
      for (int q = 0; q < P; ++q) X[q] = mk(0.f, 0.f);
    }
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const cf Z = mk(Xc[q].x + sgn * X[q].x, Xc[q].y + sgn * X[q].y);
      const cf c = cmacc(R[q], Xc[q], Z);
      const cf d = mk(__builtin_fmaf(Xc[q].x, Z.x, R[q].x), __builtin_fmaf(Xc[q].y, Z.y, R[q].y));
      R[q] = (q == SP && t == 0) ? d : c;
      Xc[q] = X[q];
    }
  }
  // Both spectra carry a factor 2 and the inverse 2 M: R -> 8 M r_xx.
  Fft<PL>::pre(R, tw, t);
  Fft<PL>::inverse(R, lds, tw, t);
  float* rl = reinterpret_cast<float*>(lds_raw);
  const float sc = 1.0f / (8.0f * (float)M);
  __syncthreads();  // every read of the exchange buffers is done
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const int n0 = 2 * (t + q * T);
    if (n0 < lmax) rl[n0] = R[q].x * sc;
    if (n0 + 1 < lmax) rl[n0 + 1] = R[q].y * sc;
  }
  __syncthreads();
  cf sv[P];
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const int n0 = 2 * (t + q * T), n1 = n0 + 1;
    const float a = n0 < lmax ? rl[n0] : (n0 > N - lmax ? rl[N - n0] : 0.f);
    const float c = n1 < lmax ? rl[n1] : (n1 > N - lmax ? rl[N - n1] : 0.f);
    sv[q] = mk(a, c);
  }
  __syncthreads();  // the windowed autocorrelation is read before the exchanges reuse the LDS
  // the taps of the first RIR are requested before the transform of s, each
  // next RIR's before the current one is transformed
  const long long r0 = ((long long)u * b.S + i) * J;
  cf Hn[kPrefetch ? P : 1];
  if constexpr (kPrefetch) load_real<PL>(Hn, A.h + uni64(b.rir_off[r0]), uni(b.rir_len[r0]), t);
  Fft<PL>::forward(sv, lds, tw, t);
  Fft<PL>::post(sv, tw, t);  // 2 S, real (s is real and even)
  for (int j = 0; j < J; ++j) {
    const long long r = r0 + j;
    cf Hv[P];
    if constexpr (kPrefetch) {
#pragma unroll
      for (int q = 0; q < P; ++q) Hv[q] = Hn[q];
      if (j + 1 < J) load_real<PL>(Hn, A.h + uni64(b.rir_off[r + 1]), uni(b.rir_len[r + 1]), t);
    } else {
      load_real<PL>(Hv, A.h + uni64(b.rir_off[r]), uni(b.rir_len[r]), t);
    }
    Fft<PL>::forward(Hv, lds, tw, t);
    Fft<PL>::post(Hv, tw, t);  // 2 H
    double part = 0.0;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const double hx = Hv[q].x, hy = Hv[q].y;
      if (q == SP && t == 0)
        part += hx * hx * (double)sv[q].x + hy * hy * (double)sv[q].y;  // bins 0 and N/2
      else
        part += 2.0 * (hx * hx + hy * hy) * (double)sv[q].x;           // bins k and N - k
    }
    const double e = block_sum_d<T>(part, s_red, t);
    if (t == 0) A.energy[r] = e / (8.0 * (double)N);
  }
}

// Source slot k of the batch: whether its descriptors are usable, whether it
// has work, its longest kept RIR, transform size and kernel family.  Slots
// without work (and unusable ones) belong to the family of the 16384-point
// transforms, which writes them.
struct EnergyItem {
  bool ok, work;
  int u, i, nx, lmax, l2, fam;
};

__device__ __forceinline__ EnergyItem energy_item(const BatchDev& b, long long k) {
  EnergyItem e;
  e.u = (int)(k / b.S);
  e.i = (int)(k - (long long)e.u * b.S);
  const int I = b.n_src[e.u], J = b.J;
  e.nx = b.src_len[e.u];
  e.lmax = 0;
  e.ok = I >= 0 && I <= b.S && e.nx >= 0;
  if (e.ok && e.i < I) {
    for (int j = 0; j < J; ++j) {
      const long long r = ((long long)e.u * b.S + e.i) * J + j;
      const int L = b.rir_len[r];
      const long long ro = b.rir_off[r];
      e.ok = e.ok && L >= 0 && ro >= 0 && ro + L <= b.h_len;
      e.lmax = L > e.lmax ? L : e.lmax;
    }
    const long long so = b.src_off[k];
    e.ok = e.ok && so >= 0 && so + e.nx <= b.x_len;
  }
  e.work = e.ok && e.i < I && e.nx > 0 && e.lmax > 0;
  e.l2 = e.work ? energy_log2n(e.lmax) : 0;
  e.fam = family_of_log2n(e.work && e.l2 <= 15 ? e.l2 : 14);
  return e;
}

// Transforms an item of family `fam` costs (half blocks, the inverse, s and
// one per mic); 1 for a slot that is only written; 0 for other families.
__device__ __forceinline__ double energy_cost(const BatchDev& b, long long k, int fam) {
  const EnergyItem e = energy_item(b, k);
  if (e.fam != fam) return 0.0;
  if (!e.work || e.l2 > 15) return 1.0;
  const int half = 1 << (e.l2 - 1);
  return (double)((e.nx + half - 1) / half + 2 + b.J);
}

// Each workgroup takes a contiguous range of the slots with about 1/G of the
// family's transforms: slot k goes to workgroup floor(G m_k / C), m_k the
// midpoint of its cost in the running sum and C the total (every workgroup
// computes the same sums).  No counter is needed, and the longest sources do
// not pile up on the workgroups that a fixed stride would give them.
// The costs are kept in `cache` (the exchange buffers, idle until the first
// transform) when the batch's slots fit it.
template <int T>
__device__ __forceinline__ void energy_range(const BatchDev& b, int fam, double* s_red, float* cache, long long cap,
                                             long long& lo, long long& hi, int t) {
  const long long items = (long long)b.U * b.S;
  const bool cached = items <= cap;
  const long long per = (items + T - 1) / T;
  const long long k0 = min(items, (long long)t * per), k1 = min(items, k0 + per);
  double c = 0.0;
  for (long long k = k0; k < k1; ++k) {
    const double ck = energy_cost(b, k, fam);
    if (cached) cache[k] = (float)ck;  // small integers: exact
    c += ck;
  }
  // inclusive scan of the per-thread sums (Hillis-Steele)
  __syncthreads();
  s_red[t] = c;
  __syncthreads();
  for (int d = 1; d < T; d <<= 1) {
    const double v = t >= d ? s_red[t - d] : 0.0;
    __syncthreads();
    s_red[t] += v;
    __syncthreads();
  }
  const double total = s_red[T - 1];
  const double base = s_red[t] - c;
  const double G = (double)gridDim.x;
  const double a = total * (double)blockIdx.x / G, z = total * (double)(blockIdx.x + 1) / G;
  // slots of this thread's chunk whose midpoint lies below a (resp. z)
  double below_a = 0.0, below_z = 0.0, p = base;
  for (long long k = k0; k < k1; ++k) {
    const double ck = cached ? (double)cache[k] : energy_cost(b, k, fam);
    const double mid = p + 0.5 * ck;
    below_a += mid < a ? 1.0 : 0.0;
    below_z += mid < z ? 1.0 : 0.0;
    p += ck;
  }
  const double na = block_sum_d<T>(below_a, s_red, t);
  const double nz = block_sum_d<T>(below_z, s_red, t);
  // every slot of positive cost has its midpoint below the total, so the
  // ranges of consecutive workgroups tile all of them
  lo = (long long)na;
  hi = (long long)nz;
}

template <int T>
__global__ __launch_bounds__(T, 2) void energy_kernel(EnergyArgs A) {
  __shared__ cf lds[max_lds_with_threads<T>()];
  __shared__ double s_red[T];
  __shared__ int s_list[T];
  __shared__ int s_n;
  const int t = threadIdx.x;
  const BatchDev& b = A.b;
  long long lo, hi;
  energy_range<T>(b, A.fam, s_red, reinterpret_cast<float*>(lds), 2LL * max_lds_with_threads<T>(), lo, hi, t);
  int err = 0;
  // The range is walked T slots at a time: the slots of this family in the
  // window are found in parallel (one per thread) and listed, so slots of
  // other families cost no serial descriptor reads.
  for (long long w = lo; w < hi; w += T) {
    __syncthreads();  // the previous window's list has been read
    if (t == 0) s_n = 0;
    __syncthreads();
    if (w + t < hi && energy_item(b, w + t).fam == A.fam) s_list[atomicAdd(&s_n, 1)] = t;
    __syncthreads();
    const int n = s_n;
    for (int q = 0; q < n; ++q) {
      const long long k = w + s_list[q];
      const EnergyItem e = energy_item(b, k);
      const int J = b.J;
      if (!e.work || e.l2 > 15) {
        // no work: 0; a bad descriptor or a kept RIR longer than 16384 taps: NaN
        const bool bad = !e.ok || e.l2 > 15;
        if (!e.ok) err |= RSIM_DEV_BADDESC;
        else if (e.l2 > 15) err |= RSIM_DEV_BADPLAN;
        for (int jj = t; jj < J; jj += T) A.energy[k * J + jj] = bad ? __builtin_nan("") : 0.0;
        continue;
      }
      const int u = __builtin_amdgcn_readfirstlane(e.u), i = __builtin_amdgcn_readfirstlane(e.i);
      const int lmax = __builtin_amdgcn_readfirstlane(e.lmax), l2 = __builtin_amdgcn_readfirstlane(e.l2);
      dispatch_plan<T>(l2, [&](auto pl) __attribute__((always_inline)) {
        using PL = decltype(pl);
        energy_source<PL>(A, u, i, lmax, lds, s_red, t);
      });
    }
  }
  if (err && t == 0) flag_status(err);
}

// ================================================================ dry power
__global__ __launch_bounds__(256) void power_kernel(BatchDev b, const float* __restrict__ x,
                                                   double* __restrict__ power) {
  __shared__ double s_d[4];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const long long n_slots = (long long)b.U * b.S;
  for (long long k = blockIdx.x; k < n_slots; k += gridDim.x) {
    const int u = (int)(k / b.S), i = (int)(k - (long long)u * b.S);
    const int I = b.n_src[u], Nx = b.src_len[u];
    const long long so = b.src_off[k];
    const bool ok = i < I && I <= b.S && Nx > 0 && so >= 0 && so + Nx <= b.x_len;
    if (!ok) {
      if (t == 0) {
        power[k] = 0.0;
        if (i < I && Nx != 0) flag_status(RSIM_DEV_BADDESC);
      }
      continue;
    }
    double acc = 0.0;
    for (int n = t; n < Nx; n += 256) {
      const double v = (double)x[so + n];
      acc += v * v;
    }
    acc = wave_sum_d(acc);
    __syncthreads();
    if (lane == 0) s_d[w] = acc;
    __syncthreads();
    if (t == 0) power[k] = ((s_d[0] + s_d[1]) + (s_d[2] + s_d[3])) / (double)Nx;
  }
}

// ========================================================= image-method RIRs
// Eq. (1): the RIR is the sum over the (2K+1)^3 images of the source in the
// mirrored rooms (a, b, c) of refl^g / d at tap ceil(d fs / c0).  One
// workgroup of 1024 threads per RIR: every image is evaluated in binary64 (no
// contraction, so each product and sum is rounded on its own, as the
// definition is written), its amplitude quantised to a multiple of 2^-40 and
// added with a 64-bit integer atomic to an LDS accumulator of kImgWindow taps
// (128 KB, the whole RIR up to 16384 taps), so the sums are exact and do not
// depend on the order of the images.  Longer RIRs are produced one window at
// a time; with more than one window, a float32 estimate of an image's
// distance (with margins far wider than its rounding) skips the windows its
// tap cannot fall in before the exact evaluation.
constexpr int kImgThreads = 1024;
constexpr int kImgWindow = 16384;
constexpr int kImgMaxOrder = 16;
constexpr int kImgMaxLen = 32768;  // taps per RIR, at most (two windows)
constexpr int kImgChunk = 4 * kImgThreads;  // slots ranked at a time

struct ImageArgs {
  const double* geom;  // [n_rir][9]: room Lx Ly Lz, source xyz, mic xyz
  const double* refl;  // [n_rir]
  float* h;
  long long h_len;
  const long long* off;
  const int* len;
  int n_rir, order, max_len;
  double fs, c0;
};

// Offset of the image in virtual room a from the microphone along one axis.
__device__ __forceinline__ double image_delta(int a, double L, double s, double m) {
#pragma clang fp contract(off)
  const double base = (a & 1) ? (L - s) : s;
  return ((double)a * L + base) - m;
}

// Sides below 10 km, source and microphone at least 5 mm inside every wall
// and 1 cm apart, refl in [0, 1] (NaN fails every test): every image is then
// at least 1 cm from the microphone.
__device__ __forceinline__ bool image_geometry_ok(const double* g, double refl) {
#pragma clang fp contract(off)
  bool ok = refl >= 0.0 && refl <= 1.0;
  for (int ax = 0; ax < 3; ++ax) {
    const double L = g[ax], s = g[3 + ax], m = g[6 + ax];
    ok = ok && L < 1e4 && s >= 0.005 && s <= L - 0.005 && m >= 0.005 && m <= L - 0.005;
  }
  const double dx = g[3] - g[6], dy = g[4] - g[7], dz = g[5] - g[8];
  return ok && ((dx * dx + dy * dy) + dz * dz) >= 1e-4;
}

// Windows [wlo, whi] an image with float32 squared-distance estimate d2f can
// reach: its tap, ceil(d fs / c0), lies within two taps of the estimate.
__device__ __forceinline__ void image_windows(float d2f, float taps_per_m, int nw, int& wlo, int& whi) {
  const float nlo = sqrtf(d2f * 0.999f) * taps_per_m - 2.0f;
  const float nhi = sqrtf(d2f * 1.001f) * taps_per_m + 2.0f;
  const float end = (float)(nw * kImgWindow);
  wlo = nlo <= 0.0f ? 0 : (nlo >= end ? nw : (int)(nlo * (1.0f / kImgWindow)));
  whi = nhi >= end ? nw - 1 : (int)(nhi * (1.0f / kImgWindow));
}

// Adds image (ia, ib, ic) to window [w0, w0 + wn) if its tap falls there.
__device__ __forceinline__ void image_add(const double (*sq)[2 * kImgMaxOrder + 1], const double* pw, int K,
                                          int ia, int ib, int ic, double fs, double c0, int w0, int wn,
                                          unsigned long long* acc) {
#pragma clang fp contract(off)
  const double d = sqrt((sq[0][ia] + sq[1][ib]) + sq[2][ic]);
  const double n = ceil((d * fs) / c0);
  if (n >= (double)w0 && n < (double)(w0 + wn)) {
    const int g = abs(ia - K) + abs(ib - K) + abs(ic - K);
    const double q = rint((pw[g] / d) * 1099511627776.0);  // 2^40
    atomicAdd(&acc[(int)n - w0], (unsigned long long)q);
  }
}

// Image v = (ia S + ib) S + ic, stepped by kImgThreads = (q2 S + q1) S + q0.
struct ImageIter {
  int ia, ib, ic;
  __device__ __forceinline__ void step(int S, int q2, int q1, int q0) {
    ic += q0;
    const int cc = ic >= S;
    ic -= cc ? S : 0;
    ib += q1 + cc;
    const int cb = ib >= S;
    ib -= cb ? S : 0;
    ia += q2 + cb;
  }
};

__global__ __launch_bounds__(kImgThreads) void image_kernel(ImageArgs A) {
#pragma clang fp contract(off)
  __shared__ unsigned long long acc[kImgWindow];
  __shared__ double sq[3][2 * kImgMaxOrder + 1];
  __shared__ float sqf[3][2 * kImgMaxOrder + 1];
  __shared__ double pw[3 * kImgMaxOrder + 1];
  __shared__ int s_list[kImgChunk];          // this workgroup's slots of the current chunk
  __shared__ int s_wcnt[kImgThreads / 64];   // nonzero slots per wave of the chunk
  const int t = threadIdx.x;
  const int K = A.order, S = 2 * K + 1, S2 = S * S, V = S2 * S;
  const int q2 = kImgThreads / S2, q1 = (kImgThreads % S2) / S, q0 = kImgThreads % S;
  const ImageIter it0{t / S2, (t % S2) / S, t % S};
  const float taps_per_m = (float)(A.fs / A.c0);
  int err = 0;
  // The slots with a nonzero length are ranked in slot order and workgroup b
  // of G takes ranks b, b + G, b + 2G, ...: every workgroup gets the same
  // number of RIRs to within one, wherever the empty slots lie (in a batch,
  // the slots of an utterance's missing sources).  Each workgroup ranks the
  // slots itself, kImgChunk at a time (four consecutive slots per thread, a
  // ballot per slot and wave, the wave counts in LDS), lists its own slots
  // of the chunk in LDS, and loads the next chunk's lengths while it makes
  // this chunk's RIRs.
  const long long G = gridDim.x, b = blockIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const unsigned long long lanes_below = (1ull << lane) - 1ull;
  int ln[4];
  for (int j = 0; j < 4; ++j) ln[j] = 4LL * t + j < A.n_rir ? A.len[4LL * t + j] : 0;
  long long base = 0;  // nonzero slots before the chunk
  for (long long c0 = 0; c0 < A.n_rir; c0 += kImgChunk) {
    __syncthreads();  // the previous chunk's list and wave counts are consumed
    int below = 0, wtot = 0;
    for (int j = 0; j < 4; ++j) {
      const unsigned long long bal = __ballot(ln[j] != 0);
      below += __popcll(bal & lanes_below);
      wtot += __popcll(bal);
    }
    if (lane == 0) s_wcnt[wv] = wtot;
    __syncthreads();
    long long pre = 0, tot = 0;
    for (int i = 0; i < kImgThreads / 64; ++i) {
      const int v = s_wcnt[i];
      pre += i < wv ? v : 0;
      tot += v;
    }
    const long long first = base + ((b - base % G) + G) % G;  // first rank >= base taken by b
    long long rank = base + pre + below;                        // of this thread's first nonzero slot
    for (int j = 0; j < 4; ++j) {
      if (ln[j] == 0) continue;
      if (rank % G == b) s_list[(rank - first) / G] = (int)(c0 + 4LL * t + j);
      ++rank;
    }
    const long long end = base + tot;
    const int mine = first < end ? (int)((end - 1 - first) / G + 1) : 0;
    base = end;
    __syncthreads();
    for (int j = 0; j < 4; ++j) {
      const long long sl = c0 + kImgChunk + 4LL * t + j;
      ln[j] = sl < A.n_rir ? A.len[sl] : 0;
    }
    for (int li = 0; li < mine; ++li) {
      const int r = uni(s_list[li]);  // the same in every lane: scalar addressing of the slot
      const int len = uni(A.len[r]);
      const long long off = uni64(A.off[r]);
      if (len < 0 || len > A.max_len || off < 0 || off + len > A.h_len) {
        err |= RSIM_DEV_BADDESC;
        continue;
      }
      if (len == 0) continue;
      const int nw = (len + kImgWindow - 1) / kImgWindow;
      const double* g = A.geom + 9LL * r;
      const double refl = A.refl[r];
      const bool ok = image_geometry_ok(g, refl);
      if (!ok) err |= RSIM_DEV_BADDESC;
      __syncthreads();  // the previous RIR's readers of the shared arrays are done
      if (t < 3 * S) {
        const int ax = t / S, a = t - ax * S - K;
        const double d = image_delta(a, g[ax], g[3 + ax], g[6 + ax]);
        sq[ax][t - ax * S] = d * d;
        sqf[ax][t - ax * S] = (float)(d * d);
      }
      if (t == 0) {
        double p = 1.0;
        for (int k = 0; k <= 3 * K; ++k) {
          pw[k] = p;
          p = p * refl;
        }
      }
      for (int wi = 0; wi < nw; ++wi) {
        const int w0 = wi * kImgWindow, wn = min(kImgWindow, len - w0);
        __syncthreads();  // the tables are written; the previous window's taps are stored
        for (int k = t; k < wn; k += kImgThreads) acc[k] = 0ull;
        __syncthreads();
        if (ok) {
          ImageIter im = it0;
          for (int v = t; v < V; v += kImgThreads) {
            bool in = true;
            if (nw > 1) {
              int wlo, whi;
              image_windows((sqf[0][im.ia] + sqf[1][im.ib]) + sqf[2][im.ic], taps_per_m, nw, wlo, whi);
              in = wlo <= wi && wi <= whi;
            }
            if (in) image_add(sq, pw, K, im.ia, im.ib, im.ic, A.fs, A.c0, w0, wn, acc);
            im.step(S, q2, q1, q0);
          }
        }
        __syncthreads();
        for (int k = t; k < wn; k += kImgThreads)
          A.h[off + w0 + k] = (float)((double)acc[k] * 9.094947017729282e-13);  // 2^-40
      }
    }
  }
  if (err && t == 0) flag_status(err);
}

// ============================================ full-length FFT filtering
// Eqs. 4-5: every signal is transformed whole, with N = 2^m >= Nx + L - 1
// points (up to 2^20), beyond what one workgroup holds in LDS.  The transform
// is split in four steps (N = N1 N2, n = N2 n1 + n2, k = k1 + N1 k2):
//   A  for every n2, the N1-point DFT over n1 of x[N2 n1 + n2], times
//      W_N^(n2 k1), stored at [k1 N2 + n2];
//   B  for every k1, the N2-point DFT over n2 of that row, stored at
//      X[k1 + N1 k2] (natural order).
// Each step is one kernel: a workgroup loads C sequences of L points (a tile
// of C L <= kFfTile complex values) into LDS, transforms them there by
// radix-4 Stockham passes (and one radix 2 when log2 L is odd: pass s with
// span Ls reads butterfly j's inputs at j + r L/R, twists them by
// W_(R Ls)^(r (j mod Ls)) and writes its outputs at
// (j - j mod Ls) R + (j mod Ls) + r Ls) and stores them, so each transform
// reads and writes global memory twice.  Real signals go in as complex with
// zero imaginary part.  Per utterance and mic the spectra are summed over
// sources (linearity), so one inverse per mic.  This is the paper's slower
// rung, kept for comparison.
constexpr int kFfThreads = 256;
constexpr int kFfStepThreads = 512;
constexpr int kFfTile = 8192;   // complex values of one workgroup's sequences
constexpr int kFfMaxL = 1024;   // points of one sequence, at most

struct FfStep {
  const cf* in;
  cf* out;
  long long sig_len;         // N: distance between consecutive signals
  int count;                 // signals
  int log2l, log2c;          // L = 2^log2l points per sequence, C = 2^log2c per workgroup
  int cols;                  // sequences per signal (a multiple of C)
  long long in_cs, in_ns;    // input (c, n) of a signal at c in_cs + n in_ns
  long long out_cs, out_ks;  // output (c, k) at c out_cs + k out_ks
  int n_fast;                // load with n varying fastest (in_ns == 1)
  int log2n, twiddle;        // outputs times W_N^(c k) when twiddle != 0
  const int* n_src;          // signals are source slots (u0 + sig / S, sig mod S): those
  int u0, S;                 // past n_src[u] are skipped (left unwritten); NULL: none
  // Fused ends (the operands of the filtering), selected per step:
  //   in_kind  0 the complex array `in`; 1 source slot (u, i) of x as real
  //            values (zero past N_x); 2 the cut RIR (u, i, j) of h (zero past
  //            L); 3 sum_i alpha_uij H[cu][i] X[cu][i] over the utterance's
  //            sources (signal = utterance cu of the chunk)
  //   out_kind 0 the complex array `out`; 1 mic j's output y_j[n] = Re / N
  //            for n < T_u (signal = utterance), out_len with mic 0
  int in_kind, out_kind, j;
  BatchDev b;
  const float* x;
  const float* h;
  const float* alpha;
  float* y;
  const cf* X;  // [chunk][S][N] source spectra
  const cf* H;  // [chunk][S][N] RIR spectra of mic j
};

template <int R, bool INV>
__device__ __forceinline__ void ff_butterfly(cf* v) {
  if constexpr (R == 2) {
    const cf a = v[0], b = v[1];
    v[0] = mk(a.x + b.x, a.y + b.y);
    v[1] = mk(a.x - b.x, a.y - b.y);
  } else {
    const cf s0 = mk(v[0].x + v[2].x, v[0].y + v[2].y), d0 = mk(v[0].x - v[2].x, v[0].y - v[2].y);
    const cf s1 = mk(v[1].x + v[3].x, v[1].y + v[3].y), d1 = mk(v[1].x - v[3].x, v[1].y - v[3].y);
    // -i d1 forward, +i d1 inverse
    const cf e1 = INV ? mk(-d1.y, d1.x) : mk(d1.y, -d1.x);
    v[0] = mk(s0.x + s1.x, s0.y + s1.y);
    v[2] = mk(s0.x - s1.x, s0.y - s1.y);
    v[1] = mk(d0.x + e1.x, d0.y + e1.y);
    v[3] = mk(d0.x - e1.x, d0.y - e1.y);
  }
}

// One radix-R Stockham pass over the C sequences in buf (sequence c, point n
// at n CP + c).  Every thread reads all its butterflies' inputs before the
// barrier and writes after it, so the pass runs in place.
template <int R, bool INV>
__device__ __forceinline__ void ff_lds_pass(cf* buf, const cf* tw, int log2l, int log2c, int CP, int Ls, int t) {
  constexpr int NB = kFfTile / R / kFfStepThreads;  // butterflies per thread, at most
  const int L = 1 << log2l, C = 1 << log2c;
  const int nb = (C * L) / R;
  const int stride = L / R;
  const int tws = L / (R * Ls);  // W_(R Ls)^e = W_L^(e tws)
  cf v[NB][R];
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    const int b = t + s * kFfStepThreads;
    if (b < nb) {
      const int c = b & (C - 1), j = b >> log2c, k = j & (Ls - 1);
#pragma unroll
      for (int r = 0; r < R; ++r) v[s][r] = buf[(j + r * stride) * CP + c];
#pragma unroll
      for (int r = 1; r < R; ++r) v[s][r] = cmul(v[s][r], tw[r * k * tws]);
      ff_butterfly<R, INV>(v[s]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NB; ++s) {
    const int b = t + s * kFfStepThreads;
    if (b < nb) {
      const int c = b & (C - 1), j = b >> log2c, k = j & (Ls - 1);
      const int base = (j - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[(base + r * Ls) * CP + c] = v[s][r];
    }
  }
  __syncthreads();
}

template <bool INV>
__global__ __launch_bounds__(kFfStepThreads) void ff_step_kernel(FfStep S) {
  __shared__ cf buf[kFfTile + kFfMaxL];  // C sequences, row stride C + 1
  __shared__ cf tw[kFfMaxL];             // W_L^m, m < L
  const int t = threadIdx.x;
  const int L = 1 << S.log2l, C = 1 << S.log2c, CP = C + 1;
  for (int m = t; m < L; m += kFfStepThreads) {
    float sn, cs;
    sincospif(2.0f * (float)m / (float)L, &sn, &cs);  // m / L exact
    tw[m] = mk(cs, INV ? sn : -sn);
  }
  const int tiles = S.cols >> S.log2c;
  const long long items = (long long)S.count * tiles;
  const float inv_n = 1.0f / (float)(1LL << S.log2n);
  for (long long it = blockIdx.x; it < items; it += gridDim.x) {
    const long long sig = it / tiles;
    const int c0 = (int)(it - sig * tiles) << S.log2c;
    if (S.n_src && (int)(sig % S.S) >= S.n_src[S.u0 + sig / S.S]) continue;  // uniform
    const BatchDev& b = S.b;
    // the signal's real input (in_kind 1, 2): values below rlen, zero after
    const float* rin = nullptr;
    long long rlen = 0;
    if (S.in_kind == 1 || S.in_kind == 2) {
      const int cu = (int)(sig / S.S), i = (int)(sig % S.S), u = S.u0 + cu;
      const bool okI = b.n_src[u] <= b.S;  // a bad count transforms zeros
      if (S.in_kind == 1) {
        const long long so = b.src_off[(long long)u * b.S + i];
        const int nx = b.src_len[u];
        if (okI && so >= 0 && nx >= 0 && so + nx <= b.x_len) {
          rin = S.x + so;
          rlen = nx;
        }
      } else {
        const long long r = ((long long)u * b.S + i) * b.J + S.j;
        const long long ro = b.rir_off[r];
        const int len = b.rir_len[r];
        if (okI && ro >= 0 && len >= 0 && ro + len <= b.h_len) {
          rin = S.h + ro;
          rlen = len;
        }
      }
    }
    const cf* src = S.in_kind == 0 ? S.in + sig * S.sig_len : nullptr;
    __syncthreads();  // the table is written; the previous tile is stored
    for (int e = t; e < C * L; e += kFfStepThreads) {
      int c, n;
      if (S.n_fast) {
        n = e & (L - 1);
        c = e >> S.log2l;
      } else {
        c = e & (C - 1);
        n = e >> S.log2c;
      }
      const long long idx = (long long)(c0 + c) * S.in_cs + (long long)n * S.in_ns;
      cf v;
      if (S.in_kind == 0) {
        v = src[idx];
      } else if (S.in_kind == 3) {
        const int cu = (int)sig, u = S.u0 + cu;
        const int I = min(b.n_src[u], b.S);
        float re = 0.f, im = 0.f;
        for (int i = 0; i < I; ++i) {
          const float a = S.alpha[((long long)u * b.S + i) * b.J + S.j];
          const long long o = ((long long)cu * b.S + i) * S.sig_len + idx;
          const cf hv = S.H[o], xv = S.X[o];
          const float pr = hv.x * xv.x - hv.y * xv.y, pi = hv.x * xv.y + hv.y * xv.x;
          re = __builtin_fmaf(a, pr, re);
          im = __builtin_fmaf(a, pi, im);
        }
        v = mk(re, im);
      } else {
        v = mk(idx < rlen ? rin[idx] : 0.f, 0.f);
      }
      buf[n * CP + c] = v;
    }
    __syncthreads();
    int Ls = 1, l = S.log2l;
    for (; l >= 2; l -= 2, Ls *= 4) ff_lds_pass<4, INV>(buf, tw, S.log2l, S.log2c, CP, Ls, t);
    if (l == 1) ff_lds_pass<2, INV>(buf, tw, S.log2l, S.log2c, CP, Ls, t);
    if (S.out_kind == 1) {
      // y_j[n] = Re(z) / N for n < T_u = Nx + Lmax - 1; an utterance whose
      // T_u exceeds N or its output stride is skipped with BADPLAN
      const int u = S.u0 + (int)sig;
      const int I = b.n_src[u], Nx = b.src_len[u];
      int lmax = 0;
      for (int i = 0; i < min(I, b.S); ++i)
        for (int jj = 0; jj < b.J; ++jj) lmax = max(lmax, b.rir_len[((long long)u * b.S + i) * b.J + jj]);
      const long long T = (I > 0 && Nx > 0 && lmax > 0) ? (long long)Nx + lmax - 1 : 0;
      const int stride = b.out_stride[u];
      const bool lead = c0 == 0 && t == 0 && S.j == 0;
      if (T > S.sig_len || T > stride) {
        if (lead) {
          flag_status(RSIM_DEV_BADPLAN);
          b.out_len[u] = 0;
        }
        continue;
      }
      if (lead) b.out_len[u] = (int)T;
      float* yj = S.y + b.out_off[u] + (long long)S.j * stride;
      for (int e = t; e < C * L; e += kFfStepThreads) {
        const int c = e & (C - 1), k = e >> S.log2c;
        const long long n = (long long)(c0 + c) * S.out_cs + (long long)k * S.out_ks;
        if (n < T) yj[n] = buf[k * CP + c].x * inv_n;
      }
      continue;
    }
    cf* dst = S.out + sig * S.sig_len + (long long)c0 * S.out_cs;
    for (int e = t; e < C * L; e += kFfStepThreads) {
      const int c = e & (C - 1), k = e >> S.log2c;
      cf z = buf[k * CP + c];
      if (S.twiddle) {
        // W_N^(n2 k1) with n2 k1 < N <= 2^20: the ratio is exact
        const float a = (float)((unsigned)(c0 + c) * (unsigned)k) * inv_n;
        float sn, cs;
        sincospif(2.0f * a, &sn, &cs);
        z = cmul(z, mk(cs, INV ? sn : -sn));
      }
      dst[(long long)c * S.out_cs + (long long)k * S.out_ks] = z;
    }
  }
}


// ================================================= FFT engine test kernels
template <class PL>
__global__ __launch_bounds__(PL::T) void rfft_kernel(const float* __restrict__ x, float* __restrict__ spec) {
  __shared__ cf lds_raw[Xch<PL>::kEntries];
  Xch<PL> lds{lds_raw, 0};
  const int t = threadIdx.x;
  const long long sig = blockIdx.x;
  const TwBase tw = Fft<PL>::bases(plan_tw<PL>(), t);
  cf v[PL::P];
  load_real<PL>(v, x + sig * PL::N, PL::N, t);
  Fft<PL>::forward(v, lds, tw, t);
  Fft<PL>::post(v, tw, t);
  cf* out = reinterpret_cast<cf*>(spec) + sig * (PL::M + 1);
#pragma unroll
  for (int q = 0; q < PL::P; ++q) {
    if (t == 0 && q == Fft<PL>::SP) {
      out[0] = mk(0.5f * v[q].x, 0.f);
      out[PL::M] = mk(0.5f * v[q].y, 0.f);
    } else {
      out[slot_bin<PL>(q, t)] = mk(0.5f * v[q].x, 0.5f * v[q].y);
    }
  }
}

template <class PL>
__global__ __launch_bounds__(PL::T) void irfft_kernel(const float* __restrict__ spec, float* __restrict__ x) {
  __shared__ cf lds_raw[Xch<PL>::kEntries];
  Xch<PL> lds{lds_raw, 0};
  const int t = threadIdx.x;
  const long long sig = blockIdx.x;
  const TwBase tw = Fft<PL>::bases(plan_tw<PL>(), t);
  const cf* in = reinterpret_cast<const cf*>(spec) + sig * (PL::M + 1);
  cf v[PL::P];
#pragma unroll
  for (int q = 0; q < PL::P; ++q) {
    if (t == 0 && q == Fft<PL>::SP) {
      v[q] = mk(2.f * in[0].x, 2.f * in[PL::M].x);
    } else {
      const cf z = in[slot_bin<PL>(q, t)];
      v[q] = mk(2.f * z.x, 2.f * z.y);
    }
  }
  Fft<PL>::pre(v, tw, t);
  Fft<PL>::inverse(v, lds, tw, t);
  const float sc = 1.0f / (float)(2 * PL::N);
  float* o = x + sig * PL::N;
#pragma unroll
  for (int r = 0; r < PL::P; ++r) {
    const int m = 2 * (t + r * PL::T);
    o[m] = v[r].x * sc;
    o[m + 1] = v[r].y * sc;
  }
}

// ======================================================= log-Mel front end
// The paper's acoustic-model features (Sec. 3): 128 log-Mel bands of 512-sample
// (32 ms) Hann windows every 160 samples (10 ms), the filterbank spanning
// 125..7500 Hz.  A workgroup holds kMelGroups groups of 32 threads, each
// group one frame through the 512-point plan (its own LDS exchange buffers;
// the plan's barriers are the workgroup's, so every group runs the same
// steps, on zeros when it has no frame).  Power |X_k|^2 goes to LDS (over the
// group's exchange buffer, free once the transform has its result in
// registers) and thread t sums bands t, t + 32, t + 64, t + 96 over their
// bins in bin order.  A thread's window samples and band weights are the same
// for every frame: they are loaded into registers once, and the band loops
// have compile-time trip counts (the widest band of each quarter), so all
// power reads of a frame are in flight together.
constexpr int kMelGroups = 2;  // one wave: its barriers cost little
constexpr int kMelChunksPerItem = 16;

struct MelArgs {
  BatchDev b;
  const float* y;
  float* feat;
  const long long* feat_off;  // [U]
  long long feat_len;
  int chunks;                 // chunks of kMelGroups frames per (utterance, mic), at most
};

__global__ __launch_bounds__(kMelGroups * 32) void logmel_kernel(MelArgs A) {
  using PL = PlanOf<9>;
  static_assert(PL::T == 32 && PL::N == kMelWin, "one 512-point plan per group of 32 threads");
  __shared__ cf lds_raw[kMelGroups][Xch<PL>::kEntries];
  static_assert(2 * Xch<PL>::kEntries >= kMelBins + kMelCapMax, "the power spectrum fits the exchange buffer");
  const int tid = threadIdx.x, grp = tid >> 5, t = tid & 31;
  float hw[2 * PL::P];
#pragma unroll
  for (int r = 0; r < PL::P; ++r) {
    hw[2 * r] = g_hann[2 * (t + r * PL::T)];
    hw[2 * r + 1] = g_hann[2 * (t + r * PL::T) + 1];
  }
  float w0[kMelCap0], w1[kMelCap1], w2[kMelCap2], w3[kMelCap3];
  int first[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) first[k] = g_mel_first[t + 32 * k];
#pragma unroll
  for (int i = 0; i < kMelCap0; ++i) w0[i] = g_mel_w[(t + 0) * kMelCapMax + i];
#pragma unroll
  for (int i = 0; i < kMelCap1; ++i) w1[i] = g_mel_w[(t + 32) * kMelCapMax + i];
#pragma unroll
  for (int i = 0; i < kMelCap2; ++i) w2[i] = g_mel_w[(t + 64) * kMelCapMax + i];
#pragma unroll
  for (int i = 0; i < kMelCap3; ++i) w3[i] = g_mel_w[(t + 96) * kMelCapMax + i];
  const BatchDev& b = A.b;
  const TwBase tw = Fft<PL>::bases(plan_tw<PL>(), t);
  float* pw = reinterpret_cast<float*>(lds_raw[grp]);
  // A work item is up to kMelChunksPerItem chunks of kMelGroups frames of one
  // (utterance, mic); the next chunk's frames load while one is transformed.
  const int per_item = (A.chunks + kMelChunksPerItem - 1) / kMelChunksPerItem;
  const long long items = (long long)b.U * b.J * per_item;
  int err = 0;
  for (long long it = blockIdx.x; it < items; it += gridDim.x) {
    const int cb = (int)(it % per_item);
    const long long uj = it / per_item;
    const int u = (int)(uj / b.J), j = (int)(uj - (long long)u * b.J);
    const int T = uni(b.out_len[u]), stride = uni(b.out_stride[u]);
    const int F = mel_frames(T), cap = mel_frames(stride);
    const int c0 = cb * kMelChunksPerItem;
    if (c0 * kMelGroups >= F) continue;
    const long long yo = uni64(b.out_off[u]) + (long long)j * stride;
    const long long fo = uni64(A.feat_off[u]);
    if (T > stride || T >= kMelMaxT || yo < 0 || yo + T > b.y_len || fo < 0 ||
        fo + (long long)b.J * cap * kMelBands > A.feat_len) {
      if (cb == 0) err |= RSIM_DEV_BADDESC;
      continue;
    }
    const int c1 = min(c0 + kMelChunksPerItem, (F + kMelGroups - 1) / kMelGroups);
    // One buffer resource for the mic's signal, the same for both groups of
    // the wave (a per-group base would make the compiler serialise every
    // load over the groups); a frame is a lane offset into it.  A group
    // without a frame reads frame 0 (in range, results unused).
    const rsrc_t ys = make_rsrc(A.y + yo, T * 4);
    auto load_frame = [&](cf* dst, int fr) __attribute__((always_inline)) {
      const int vo = opaque_v((fr < F ? fr * kMelHop * 4 : 0) + 8 * t);
#pragma unroll
      for (int r = 0; r < PL::P; ++r) dst[r] = ld2(ys, vo, 8 * r * PL::T);
    };
    cf vn[PL::P];
    load_frame(vn, c0 * kMelGroups + grp);
    for (int c = c0; c < c1; ++c) {
      const int fr = c * kMelGroups + grp;
      const bool live = fr < F;
      cf v[PL::P];
#pragma unroll
      for (int r = 0; r < PL::P; ++r) v[r] = mk(vn[r].x * hw[2 * r], vn[r].y * hw[2 * r + 1]);
      if (c + 1 < c1) load_frame(vn, fr + kMelGroups);
      __syncthreads();  // the previous chunk's band sums have read pw
      Xch<PL> lds{lds_raw[grp], 0};
      Fft<PL>::forward(v, lds, tw, t);
      Fft<PL>::post(v, tw, t);  // 2 X
      __syncthreads();  // every exchange read is done before pw overwrites the buffer
#pragma unroll
      for (int q = 0; q < PL::P; ++q) {
        if (t == 0 && q == Fft<PL>::SP) {
          pw[0] = 0.25f * v[q].x * v[q].x;
          pw[PL::M] = 0.25f * v[q].y * v[q].y;
        } else {
          pw[slot_bin<PL>(q, t)] = 0.25f * (v[q].x * v[q].x + v[q].y * v[q].y);
        }
      }
      __syncthreads();
      if (live) {
        float* out = A.feat + fo + ((long long)j * cap + fr) * kMelBands;
        const float m0 = mel_band<kMelCap0>(w0, pw, first[0]);
        const float m1 = mel_band<kMelCap1>(w1, pw, first[1]);
        const float m2 = mel_band<kMelCap2>(w2, pw, first[2]);
        const float m3 = mel_band<kMelCap3>(w3, pw, first[3]);
        out[t] = logf(m0 + 1e-6f);
        out[t + 32] = logf(m1 + 1e-6f);
        out[t + 64] = logf(m2 + 1e-6f);
        out[t + 96] = logf(m3 + 1e-6f);
      }
    }
  }
  if (err && tid == 0) flag_status(err);
}


// ================================================================ host side
template <class PL>
static void fill_plan(std::vector<float2>& tw, int base) {
  auto W = [](long long e, long long n) {
    e %= n;
    const double a = -2.0 * 3.14159265358979323846264338327950288 * (double)e / (double)n;
    return make_float2((float)std::cos(a), (float)std::sin(a));
  };
  for (int p = 1; p <= PL::NP - 2; ++p) {
    const int R = PL::R[p], Ls = PL::ls(p);
    for (int r = 0; r < R; ++r)
      for (int k = 0; k < Ls; ++k) tw[base + PL::mid_off(p) + r * Ls + k] = W((long long)r * k, (long long)R * Ls);
  }
  for (int r = 0; r < PL::RL; ++r)
    for (int k = 0; k <= PL::T; ++k) tw[base + PL::LAST_OFF + r * (PL::T + 1) + k] = W((long long)r * k, PL::M);
  for (int q = 0; q < PL::RL; ++q)
    for (int c = 0; c <= PL::T; ++c)
      tw[base + PL::POST_OFF + q * (PL::T + 1) + c] = W((long long)c + 2LL * PL::T * q, PL::N);
}

void fill_twiddles(float* out) {
  std::vector<float2> tw(kTwTotal, make_float2(0.f, 0.f));
  sfor<kNumSizes>([&](auto c) {
    constexpr int l2 = kMinL2 + decltype(c)::value;
    fill_plan<PlanOf<l2>>(tw, tw_off<l2>());
  });
  std::memcpy(out, tw.data(), sizeof(float2) * kTwTotal);
}

// Single-utterance descriptor arrays live at the head of the ola workspace.
struct OlaDesc {
  int n_src, src_len, rir_len0, rir_len, out_stride, out_len, log2n, hop;
  long long src_off, rir_off, out_off;
  float alpha;
};

__global__ void ola_setup_kernel(OlaDesc* d, int nx, int nh, int l2, int hop) {
  d->n_src = 1;
  d->src_len = nx;
  d->rir_len0 = nh;
  d->rir_len = nh;
  d->out_stride = nx + nh - 1;
  d->out_len = 0;
  d->log2n = l2;
  d->hop = hop;
  d->src_off = 0;
  d->rir_off = 0;
  d->out_off = 0;
  d->alpha = 1.0f;
}

}  // namespace rsim

using namespace rsim;

// Scratch of rsim_simulate_static, for callers that cannot allocate: one copy
// per device, held from the library's load on that device until the process
// ends.  Host code never passes this name to a kernel (on the host it is a
// stand-in, not a device address); init looks up each device's address with
// hipGetSymbolAddress and the calls use that.
static __device__ __align__(256) unsigned char scratch[RSIM_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kFamT[kNumFam] = {32, 64, 128, 256, 512, 1024};
// Kernel variants: (mic accumulators JG, waves per SIMD the registers are
// sized for).  0: JG 1 / 2 waves, 1: JG 2 / 1 wave, 2: JG 2 / 2 waves,
// 3: JG 1 / 4 waves (with one exchange buffer, so the LDS admits them).  A
// tune table names one per family (code = index + 1).
constexpr int kNumVar = 4;
constexpr int kVarJG[kNumVar] = {1, 2, 2, 1};
constexpr int kFamMaxM[kNumFam] = {max_m_with_threads<32>(),  max_m_with_threads<64>(),
                                   max_m_with_threads<128>(), max_m_with_threads<256>(),
                                   max_m_with_threads<512>(), max_m_with_threads<1024>()};
constexpr int kFamOrder[kNumFam] = {4, 5, 3, 2, 1, 0};  // launch order: the common sizes first
constexpr int kMaxDev = 64;

struct DevState {
  bool init = false;
  int cus = 0;
  int occ[kNumVar][kNumFam] = {};  // [variant][family]
  int occ_bwd[kNumFam] = {};
  int occ_feat[kNumFam] = {};  // mix kernels with the fused front end (families 2-4)
  // Side streams (default priority) and events that let the family kernels
  // of one call run concurrently: the tail of one family overlaps the next.
  static constexpr int kSide = kNumFam;  // a call issues at most kNumFam + 1 parallel kernels
  hipStream_t side[kSide] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kSide] = {};
  // This device's copy of `scratch` (rsim_simulate_static's workspace).
  void* static_ws = nullptr;
};

std::mutex g_mu;
DevState g_dev[kMaxDev];

struct Retired {
  hipGraphExec_t exec;
  hipEvent_t done;
  bool seen_done;  // its event was observed complete by an earlier pass
};
std::deque<Retired> g_retired;


template <int JG, int MINW>
const void* mix_kernel_ptr_v(int fam) {
  switch (fam) {
    case 0: return reinterpret_cast<const void*>(&mix_kernel<32, JG, MINW>);
    case 1: return reinterpret_cast<const void*>(&mix_kernel<64, JG, MINW>);
    case 2: return reinterpret_cast<const void*>(&mix_kernel<128, JG, MINW>);
    case 3: return reinterpret_cast<const void*>(&mix_kernel<256, JG, MINW>);
    case 4: return reinterpret_cast<const void*>(&mix_kernel<512, JG, MINW>);
    // 1024 threads leave 128 registers per thread: one mic accumulator
    default: return reinterpret_cast<const void*>(&mix_kernel<1024, 1, 4>);
  }
}
const void* bwd_kernel_ptr(int fam) {
  switch (fam) {
    case 0: return reinterpret_cast<const void*>(&bwd_kernel<32>);
    case 1: return reinterpret_cast<const void*>(&bwd_kernel<64>);
    case 2: return reinterpret_cast<const void*>(&bwd_kernel<128>);
    case 3: return reinterpret_cast<const void*>(&bwd_kernel<256>);
    case 4: return reinterpret_cast<const void*>(&bwd_kernel<512>);
    default: return reinterpret_cast<const void*>(&bwd_kernel<1024>);
  }
}
const void* bwd_rir_kernel_ptr(int fam) {
  switch (fam) {
    case 0: return reinterpret_cast<const void*>(&bwd_rir_kernel<32>);
    case 1: return reinterpret_cast<const void*>(&bwd_rir_kernel<64>);
    case 2: return reinterpret_cast<const void*>(&bwd_rir_kernel<128>);
    case 3: return reinterpret_cast<const void*>(&bwd_rir_kernel<256>);
    case 4: return reinterpret_cast<const void*>(&bwd_rir_kernel<512>);
    default: return reinterpret_cast<const void*>(&bwd_rir_kernel<1024>);
  }
}
const void* energy_kernel_ptr(int fam) {
  switch (fam) {
    case 0: return reinterpret_cast<const void*>(&energy_kernel<32>);
    case 1: return reinterpret_cast<const void*>(&energy_kernel<64>);
    case 2: return reinterpret_cast<const void*>(&energy_kernel<128>);
    case 3: return reinterpret_cast<const void*>(&energy_kernel<256>);
    case 4: return reinterpret_cast<const void*>(&energy_kernel<512>);
    default: return reinterpret_cast<const void*>(&energy_kernel<1024>);
  }
}
const void* mix_rir_kernel_ptr(int fam) {
  switch (fam) {
    case 0: return reinterpret_cast<const void*>(&mix_rir_kernel<32>);
    case 1: return reinterpret_cast<const void*>(&mix_rir_kernel<64>);
    case 2: return reinterpret_cast<const void*>(&mix_rir_kernel<128>);
    case 3: return reinterpret_cast<const void*>(&mix_rir_kernel<256>);
    case 4: return reinterpret_cast<const void*>(&mix_rir_kernel<512>);
    default: return reinterpret_cast<const void*>(&mix_rir_kernel<1024>);
  }
}
const void* bwd_finish_kernel_ptr(int fam) {
  switch (fam) {
    case 0: return reinterpret_cast<const void*>(&bwd_finish_kernel<32>);
    case 1: return reinterpret_cast<const void*>(&bwd_finish_kernel<64>);
    case 2: return reinterpret_cast<const void*>(&bwd_finish_kernel<128>);
    case 3: return reinterpret_cast<const void*>(&bwd_finish_kernel<256>);
    case 4: return reinterpret_cast<const void*>(&bwd_finish_kernel<512>);
    default: return reinterpret_cast<const void*>(&bwd_finish_kernel<1024>);
  }
}
// Families with a fused front-end kernel (N = 4096, 8192, 16384), and its
// variant (two mics per pass, registers for one wave per SIMD).
constexpr bool feat_family(int fam) { return fam >= 2 && fam <= 4; }
constexpr int kFeatVar = 1;
const void* mix_feat_kernel_ptr(int fam) {
  switch (fam) {
    case 2: return reinterpret_cast<const void*>(&mix_kernel<128, 2, 1, true>);
    case 3: return reinterpret_cast<const void*>(&mix_kernel<256, 2, 1, true>);
    case 4: return reinterpret_cast<const void*>(&mix_kernel<512, 2, 1, true>);
    default: return nullptr;
  }
}
const void* mix_kernel_ptr(int fam, int var) {
  switch (var) {
    case 0: return mix_kernel_ptr_v<1, 2>(fam);
    case 1: return mix_kernel_ptr_v<2, 1>(fam);
    case 2: return mix_kernel_ptr_v<2, 2>(fam);
    default: return mix_kernel_ptr_v<1, 4>(fam);
  }
}

// Variant of a family when the tune table names none: two mic accumulators
// for every family but the 1024-thread one, which has a single variant.
constexpr int kDefaultVar = 1;
constexpr int kFam1024Var = 3;
// Mic accumulators of family f's kernel.
int mic_group(int f, const TuneDev& td) { return kVarJG[td.variant[f]]; }

// The log-Mel tables in binary64, rounded once to float32: the periodic Hann
// window and, per band b, the nonzero weights of the triangle over the Mel
// edges b, b+1, b+2 (130 edges equally spaced in m(f) = 2595 log10(1 + f/700)
// from 125 to 7500 Hz) at the bin frequencies k * 16000 / 512.
bool upload_mel_tables() {
  std::vector<float> hann(kMelWin);
  for (int n = 0; n < kMelWin; ++n) hann[n] = (float)(0.5 - 0.5 * std::cos(2.0 * M_PI * n / kMelWin));
  auto mel = [](double f) { return 2595.0 * std::log10(1.0 + f / 700.0); };
  auto hz = [](double m) { return 700.0 * (std::pow(10.0, m / 2595.0) - 1.0); };
  double edges[kMelBands + 2];
  const double m0 = mel(125.0), m1 = mel(7500.0);
  for (int e = 0; e < kMelBands + 2; ++e)
    edges[e] = e == kMelBands + 1 ? hz(m1) : hz(m0 + (m1 - m0) * e / (double)(kMelBands + 1));
  int first[kMelBands], count[kMelBands];
  std::vector<float> w((size_t)kMelBands * kMelCapMax, 0.f);
  for (int b = 0; b < kMelBands; ++b) {
    const double lo = edges[b], c = edges[b + 1], hi = edges[b + 2];
    first[b] = 0;
    count[b] = 0;
    for (int k = 0; k < kMelBins; ++k) {
      const double f = k * 16000.0 / kMelWin;
      const double v = std::max(0.0, std::min((f - lo) / (c - lo), (hi - f) / (hi - c)));
      if (v > 0.0) {
        if (count[b] == 0) first[b] = k;
        // the weights of a band are consecutive bins
        if (count[b] != k - first[b] || count[b] >= mel_cap(b / 32)) return false;
        w[(size_t)b * kMelCapMax + count[b]] = (float)v;
        ++count[b];
      }
    }
  }
  return hipMemcpyToSymbol(HIP_SYMBOL(g_hann), hann.data(), sizeof(float) * kMelWin) == hipSuccess &&
         hipMemcpyToSymbol(HIP_SYMBOL(g_mel_first), first, sizeof(first)) == hipSuccess &&
         hipMemcpyToSymbol(HIP_SYMBOL(g_mel_w), w.data(), sizeof(float) * w.size()) == hipSuccess;
}

rsim_status init_locked(int dev) {
  DevState& st = g_dev[dev];
  if (st.init) return RSIM_OK;
  std::vector<float> tw(2 * (size_t)kTwTotal);
  fill_twiddles(tw.data());
  if (hipMemcpyToSymbol(HIP_SYMBOL(g_tw), tw.data(), sizeof(float) * tw.size()) != hipSuccess)
    return RSIM_EDEVICE;
  const int zero = 0;
  if (hipMemcpyToSymbol(HIP_SYMBOL(g_status), &zero, sizeof(int)) != hipSuccess) return RSIM_EDEVICE;
  if (!upload_mel_tables()) return RSIM_EDEVICE;
  if (hipDeviceGetAttribute(&st.cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return RSIM_EDEVICE;
  for (int v = 0; v < kNumVar; ++v)
    for (int f = 0; f < kNumFam; ++f) {
      int n = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, mix_kernel_ptr(f, v), kFamT[f], 0) !=
          hipSuccess)
        return RSIM_EDEVICE;
      st.occ[v][f] = n > 0 ? n : 1;
    }
  for (int f = 0; f < kNumFam; ++f) {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, bwd_kernel_ptr(f), kFamT[f], 0) != hipSuccess)
      return RSIM_EDEVICE;
    st.occ_bwd[f] = n > 0 ? n : 1;
    if (feat_family(f)) {
      n = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, mix_feat_kernel_ptr(f), kFamT[f], 0) != hipSuccess)
        return RSIM_EDEVICE;
      st.occ_feat[f] = n > 0 ? n : 1;
    }
  }
  if (!st.fork) {
    if (hipEventCreateWithFlags(&st.fork, hipEventDisableTiming) != hipSuccess) return RSIM_EDEVICE;
    for (int k = 0; k < DevState::kSide; ++k) {
      if (hipStreamCreateWithFlags(&st.side[k], hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&st.join[k], hipEventDisableTiming) != hipSuccess)
        return RSIM_EDEVICE;
    }
  }
  if (!st.static_ws) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RSIM_EDEVICE;
    st.static_ws = p;
  }
  if (hipDeviceSynchronize() != hipSuccess) return RSIM_EDEVICE;
  st.init = true;
  return RSIM_OK;
}

rsim_status ensure_init(hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return RSIM_EDEVICE;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_dev[dev].init) return RSIM_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (s && hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return RSIM_ENOTINIT;
  return init_locked(dev);
}

const DevState& dev_state() {
  static const DevState none;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return none;
  return g_dev[dev];
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// A failed HIP call leaves a sticky "last error" that the caller's next
// runtime check (torch's included) would report as its own: clear it.
rsim_status clear_error(rsim_status st) {
  (void)hipGetLastError();
  return st;
}

TuneDev default_tune() {
  TuneDev t;
  for (int m = 9; m <= 15; ++m) {
    const double N = double(1 << m);
    t.cost_fft[m - 9] = (float)(2.5 * N * m);
    t.cost_mac[m - 9] = (float)(8.0 * (N / 2 + 1));
  }
  t.one_size = 1;
  for (int f = 0; f < kNumFam; ++f) t.variant[f] = f == kNumFam - 1 ? kFam1024Var : kDefaultVar;
  return t;
}

// The tune table of the fused front end: only the sizes with a fused kernel
// (N = 4096, 8192, 16384) stay enabled, each family with its one variant.
TuneDev feat_tune(const rsim_tune* tune);

// A tune table is valid when every cost is finite and non-negative and every
// variant code is 0 (the default) or 1..4.
bool tune_ok(const rsim_tune* tune) {
  if (!tune) return true;
  for (int k = 0; k < 7; ++k)
    if (!std::isfinite(tune->cost_fft[k]) || tune->cost_fft[k] < 0.f || !std::isfinite(tune->cost_mac[k]) ||
        tune->cost_mac[k] < 0.f)
      return false;
  for (int f = 0; f < kNumFam; ++f)
    if (tune->variant[f] < 0 || tune->variant[f] > kNumVar) return false;
  return true;
}

TuneDev to_dev(const rsim_tune* tune) {
  TuneDev t = default_tune();
  if (!tune) return t;
  for (int k = 0; k < 7; ++k) {
    t.cost_fft[k] = tune->cost_fft[k];
    t.cost_mac[k] = tune->cost_mac[k];
  }
  t.one_size = tune->one_size;
  for (int f = 0; f < kNumFam - 1; ++f)
    if (tune->variant[f] > 0) t.variant[f] = tune->variant[f] - 1;
  return t;
}

TuneDev feat_tune(const rsim_tune* tune) {
  TuneDev td = to_dev(tune);
  for (int m = 9; m <= 15; ++m)
    if (!feat_family(family_of_log2n(m))) td.cost_fft[m - 9] = td.cost_mac[m - 9] = 0.f;
  for (int f = 0; f < kNumFam; ++f)
    if (feat_family(f)) td.variant[f] = kFeatVar;
  return td;
}
constexpr int kFeatSizeBits = (1 << 12) | (1 << 13) | (1 << 14);

// Families that may receive work.
void families_used(const rsim_batch* b, const TuneDev& td, bool used[kNumFam]) {
  for (int f = 0; f < kNumFam; ++f) used[f] = false;
  for (int m = 9; m <= 15; ++m) {
    const bool on = b->fft_log2n ? (b->fft_sizes == 0 || ((b->fft_sizes >> m) & 1)) : td.cost_fft[m - 9] > 0.f;
    if (on) used[family_of_log2n(m)] = true;
  }
}

struct WsLayout {
  size_t hdr, sched, lists, costs, scratch, total;
  int gsplit[kNumFam];          // forward: work items per utterance (mic groups)
  int psplit[kNumFam];          // forward: block ranges per (utterance, mic group)
  size_t fam_seam[kNumFam];     // forward: byte offset of each family's seam buffers (psplit > 1)
  int nsplit;                   // adjoint: parts per utterance
  size_t fam_partial[kNumFam];  // adjoint: byte offset of each family's part spectra (nsplit > 1)
  size_t fam_hspec[kNumFam];    // adjoint: byte offset of each family's shared RIR spectra (nsplit > 1)
  size_t fam_scratch[kNumFam];  // byte offset of each family's slots (families run concurrently)
  long long slot_cf[kNumFam];
  int grid[kNumFam];
};

// A data array may be NULL when its length is 0: nothing of it is then read
// or written (every access is bounded by descriptors checked against that
// length).
bool arr_ok(const void* p, long long len) { return p != nullptr || len == 0; }

bool batch_ok(const rsim_batch* b) {
  if (!b || b->n_utt < 0 || b->n_mic < 1 || b->max_src < 1 || b->max_rir_len0 < 0) return false;
  if (b->x_len < 0 || b->h_len < 0 || b->y_len < 0) return false;
  if (b->n_utt == 0) return true;
  return b->n_src && b->src_len && b->src_off && b->rir_off && b->rir_len0 && b->rir_len &&
         b->out_off && b->out_stride && b->out_len;
}

// Workspace layout of a call.  cap > 0 (forward only) bounds the total: when
// the persistent grids' scratch slots do not fit, every used family's grid is
// shrunk in proportion (at least one workgroup each; the kernels pop work
// items until their list is empty, so any grid size is correct).  The result
// then has total > cap only when even that does not fit.
WsLayout layout(const rsim_batch* b, const TuneDev& td, bool backward, const DevState& st, size_t cap = 0,
                bool feat = false) {
  WsLayout L;
  const size_t U = (size_t)b->n_utt;
  L.hdr = 0;
  L.sched = align256(sizeof(WsHeader));
  L.lists = L.sched + align256(U * sizeof(Sched));
  L.costs = L.lists + align256((size_t)kNumFam * U * sizeof(int));
  L.scratch = L.costs + align256(U * 8 * sizeof(float));
  bool used[kNumFam];
  families_used(b, td, used);
  const long long S = b->max_src, J = b->n_mic;
  // Without a device (size queries on a host) assume 256 CUs.
  const int cus = st.cus > 0 ? st.cus : 256;
  // The adjoint splits utterances into parts when there are fewer of them
  // than compute units (each part recomputes the RIR spectra).
  L.nsplit = 1;
  if (backward && U > 0 && (size_t)cus > U) L.nsplit = (int)std::min<size_t>(4, (cus + U - 1) / U);
  size_t off = L.scratch;
  for (int f = 0; f < kNumFam; ++f) {
    const long long M = kFamMaxM[f];
    // The forward splits utterances by mic group when there are fewer of
    // them than compute units (each group then transforms the sources itself).
    const int ngf = (int)((J + mic_group(f, td) - 1) / mic_group(f, td));
    L.gsplit[f] = !backward && U > 0 && (size_t)cus > U && ngf > 1 ? ngf : 1;
    // With fewer than four work items per compute unit, each (utterance, mic
    // group) is split into block ranges too (up to 16, one per block at
    // most), so that the longest utterances no longer set the tail of the
    // launch: its RIR spectra then come from a pass of their own and the
    // work items need no scratch slot.  (One GPU's eighth of the batched
    // epoch, 256 utterances: 0.83 ms unsplit, 0.69 ms splitting below two
    // items per CU, 0.58 ms below four.)  Not with a cap on the workspace
    // (the allocation-free entry keeps the smaller footprint of the unsplit
    // form) nor with the fused front end.
    L.psplit[f] = 1;
    if (!backward && !feat && cap == 0 && U > 0) {
      const size_t base_items = U * (size_t)L.gsplit[f], want = 4 * (size_t)cus;
      if (base_items < want) L.psplit[f] = (int)std::min<size_t>(16, (want + base_items - 1) / base_items);
    }
    const size_t items = U * (size_t)(backward ? L.nsplit : L.gsplit[f] * L.psplit[f]);
    // forward slot: the RIR spectra (unless split: shared buffer) and, when
    // one work item runs several mic groups, the block's source spectra
    const long long spectra =
        backward ? (2 * S * J + 2 * J)
                 : (L.psplit[f] > 1 ? 0 : S * J) + (J > mic_group(f, td) && L.gsplit[f] == 1 ? S : 0);
    // the fused front end's two overlap-add accumulators of 2 M samples per mic
    L.slot_cf[f] = spectra * M + (feat ? 2 * J * M : 0);
    // the largest occupancy used without a device; at most 8 workgroups per
    // CU and one per work item
    int occ = st.init ? (backward ? st.occ_bwd[f] : feat ? st.occ_feat[f] : st.occ[td.variant[f]][f]) : 8;
    if (occ > 8) occ = 8;
    long long g = (long long)cus * occ;
    if (g > (long long)items) g = (long long)items;
    if (g < 1) g = 1;
    L.grid[f] = (int)g;
  }
  // the block split's shared RIR spectra and seam buffers (fixed sizes)
  size_t split_bytes = 0;
  for (int f = 0; f < kNumFam; ++f)
    if (used[f] && !backward && L.psplit[f] > 1)
      split_bytes += align256(U * (size_t)(S * J) * (size_t)kFamMaxM[f] * sizeof(cf)) +
                     align256(U * (size_t)L.psplit[f] * (size_t)J * (size_t)kFamMaxM[f] * sizeof(float));
  if (cap > 0 && !backward) {
    size_t want = 0;
    for (int f = 0; f < kNumFam; ++f)
      if (used[f]) want += align256((size_t)L.grid[f] * (size_t)L.slot_cf[f] * sizeof(cf));
    if (off + split_bytes + want > cap) {
      const size_t room = cap > off + split_bytes ? cap - off - split_bytes : 0;
      for (int f = 0; f < kNumFam; ++f) {
        if (!used[f]) continue;
        const size_t per = (size_t)L.slot_cf[f] * sizeof(cf);
        const size_t mine = align256((size_t)L.grid[f] * per);
        // the family's share of the room, less the alignment padding, so
        // that the shares' aligned sizes add up to at most the room
        size_t share = (size_t)((long double)room * (long double)mine / (long double)want);
        share = share > 256 ? share - 256 : 0;
        const long long g = per ? (long long)(share / per) : L.grid[f];
        L.grid[f] = (int)std::max(1LL, std::min<long long>(g, L.grid[f]));
      }
    }
  }
  for (int f = 0; f < kNumFam; ++f) {
    L.fam_scratch[f] = off;
    if (used[f]) off += align256((size_t)L.grid[f] * (size_t)L.slot_cf[f] * sizeof(cf));
  }
  for (int f = 0; f < kNumFam; ++f) {
    const bool split = backward ? L.nsplit > 1 : L.psplit[f] > 1;
    L.fam_partial[f] = off;
    if (used[f] && backward && L.nsplit > 1)
      off += align256(U * (size_t)L.nsplit * (size_t)(S * J) * (size_t)kFamMaxM[f] * sizeof(cf));
    L.fam_hspec[f] = off;
    if (used[f] && split) off += align256(U * (size_t)(S * J) * (size_t)kFamMaxM[f] * sizeof(cf));
    L.fam_seam[f] = off;
    if (used[f] && !backward && L.psplit[f] > 1)
      off += align256(U * (size_t)L.psplit[f] * (size_t)J * (size_t)kFamMaxM[f] * sizeof(float));
  }
  L.total = off;
  return L;
}

BatchDev to_dev(const rsim_batch* b) {
  BatchDev d;
  d.U = b->n_utt;
  d.J = b->n_mic;
  d.S = b->max_src;
  d.x_len = b->x_len;
  d.h_len = b->h_len;
  d.y_len = b->y_len;
  d.n_src = b->n_src;
  d.src_len = b->src_len;
  d.src_off = reinterpret_cast<const long long*>(b->src_off);
  d.rir_off = reinterpret_cast<const long long*>(b->rir_off);
  d.rir_len0 = b->rir_len0;
  d.rir_len = b->rir_len;
  d.out_off = reinterpret_cast<const long long*>(b->out_off);
  d.out_stride = b->out_stride;
  d.out_len = b->out_len;
  d.order = b->order;
  d.fft_log2n = b->fft_log2n;
  d.hop = b->hop;
  d.fft_sizes = b->fft_sizes;
  return d;
}

// The kernels of one call, recorded as data so that they can be issued on
// streams or built into a graph: an optional cut, the schedule, then one
// persistent kernel per FFT-size family (independent of each other).
struct Node {
  const void* fn = nullptr;
  dim3 grid, block;
  alignas(16) unsigned char arg[512];
  void* params[1];
  template <class A>
  void set(const void* f, dim3 g, dim3 bl, const A& a) {
    static_assert(sizeof(A) <= sizeof(arg), "kernel argument block too large");
    fn = f;
    grid = g;
    block = bl;
    std::memcpy(arg, &a, sizeof(A));
  }
  void** p() {
    params[0] = arg;
    return params;
  }
};

struct CallPlan {
  bool has_gen = false;  // image-method RIRs before the cut
  Node gen;
  bool has_cut = false;
  Node cut, prep, sched;
  Node fam[kNumFam + 1];  // the family kernels (and, for the adjoint, the zero fill)
  // Optional kernels before and after fam[k] on its stream (the adjoint's
  // RIR spectra and finishing pass of a family).
  Node pre[kNumFam + 1], post[kNumFam + 1];
  bool has_pre[kNumFam + 1] = {}, has_post[kNumFam + 1] = {};
  int nf = 0;
};

bool capturing(hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (!s) return false;
  return hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// Issues the plan on s.  Several families run concurrently on the library's
// side streams (forked from s after the schedule and joined back into s),
// each with its kernels before and after it on the same stream; when s is
// being captured by the caller they run one after the other on s.
rsim_status issue_eager(CallPlan& P, hipStream_t s) {
  const DevState& st = dev_state();
  if (P.has_gen && hipLaunchKernel(P.gen.fn, P.gen.grid, P.gen.block, P.gen.p(), 0, s) != hipSuccess)
    return RSIM_EDEVICE;
  if (P.has_cut && hipLaunchKernel(P.cut.fn, P.cut.grid, P.cut.block, P.cut.p(), 0, s) != hipSuccess)
    return RSIM_EDEVICE;
  if (hipLaunchKernel(P.prep.fn, P.prep.grid, P.prep.block, P.prep.p(), 0, s) != hipSuccess)
    return RSIM_EDEVICE;
  if (hipLaunchKernel(P.sched.fn, P.sched.grid, P.sched.block, P.sched.p(), 0, s) != hipSuccess)
    return RSIM_EDEVICE;
  static_assert(sizeof(P.fam) / sizeof(P.fam[0]) <= DevState::kSide + 1, "one side stream per extra kernel");
  const bool fork = P.nf > 1 && st.fork && !capturing(s);
  // The fork/join events are shared device state: serialise their use.
  std::unique_lock<std::mutex> lk(g_mu, std::defer_lock);
  if (fork) {
    lk.lock();
    if (hipEventRecord(st.fork, s) != hipSuccess) return RSIM_EDEVICE;
  }
  for (int k = 0; k < P.nf; ++k) {
    hipStream_t fs = s;
    if (fork && k > 0) {
      fs = st.side[k - 1];
      if (hipStreamWaitEvent(fs, st.fork, 0) != hipSuccess) return RSIM_EDEVICE;
    }
    if (P.has_pre[k]) {
      Node& pn = P.pre[k];
      if (hipLaunchKernel(pn.fn, pn.grid, pn.block, pn.p(), 0, fs) != hipSuccess) return RSIM_EDEVICE;
    }
    Node& n = P.fam[k];
    if (hipLaunchKernel(n.fn, n.grid, n.block, n.p(), 0, fs) != hipSuccess) return RSIM_EDEVICE;
    if (P.has_post[k]) {
      Node& qn = P.post[k];
      if (hipLaunchKernel(qn.fn, qn.grid, qn.block, qn.p(), 0, fs) != hipSuccess) return RSIM_EDEVICE;
    }
    if (fork && k > 0) {
      if (hipEventRecord(st.join[k - 1], fs) != hipSuccess ||
          hipStreamWaitEvent(s, st.join[k - 1], 0) != hipSuccess)
        return RSIM_EDEVICE;
    }
  }
  return RSIM_OK;
}

// Executable graphs are destroyed late: one whose completion event has been
// seen complete is destroyed only at a later call (two-phase), never in the
// same pass that observed it.
void gc_retired(bool wait) {
  while (!g_retired.empty()) {
    Retired& r = g_retired.front();
    if (wait) {
      (void)hipEventSynchronize(r.done);
    } else if (!r.seen_done) {
      break;
    }
    (void)hipGraphExecDestroy(r.exec);
    (void)hipEventDestroy(r.done);
    g_retired.pop_front();
  }
  if (!wait) {
    for (Retired& r : g_retired) {
      if (r.seen_done) continue;
      const hipError_t q = hipEventQuery(r.done);
      if (q == hipErrorNotReady) {
        (void)hipGetLastError();  // not an error: leave none behind
        break;
      }
      if (q == hipSuccess) r.seen_done = true;
      else break;
    }
  }
}

// Builds the plan into a graph (a chain: cut -> schedule -> each family's
// kernels), instantiates it and launches it on s.  The graph is
// built node by node, not captured, so no stream other than s is involved.
// The executable graph is destroyed once an event recorded after its launch
// has completed.
rsim_status issue_graph(CallPlan& P, hipStream_t s) {
  if (capturing(s)) return RSIM_EINVAL;
  hipGraph_t g = nullptr;
  if (hipGraphCreate(&g, 0) != hipSuccess) return RSIM_EDEVICE;
  auto add = [&](Node& n, const hipGraphNode_t* deps, size_t nd, hipGraphNode_t* out) {
    hipKernelNodeParams kp;
    std::memset(&kp, 0, sizeof(kp));
    kp.func = const_cast<void*>(n.fn);
    kp.gridDim = n.grid;
    kp.blockDim = n.block;
    kp.sharedMemBytes = 0;
    kp.kernelParams = n.p();
    kp.extra = nullptr;
    return hipGraphAddKernelNode(out, g, deps, nd, &kp) == hipSuccess;
  };
  // A chain: cut -> schedule -> family kernels one after another.  Graphs
  // with parallel branches are not built: a run with them ended in a host
  // segmentation fault whose cause is not identified (concurrent family
  // kernels remain available on the eager path).
  hipGraphNode_t prev = nullptr;
  bool ok = true;
  if (P.has_gen) ok = add(P.gen, nullptr, 0, &prev);
  if (ok && P.has_cut) {
    hipGraphNode_t cn = nullptr;
    ok = add(P.cut, prev ? &prev : nullptr, prev ? 1 : 0, &cn);
    prev = cn;
  }
  hipGraphNode_t node = nullptr;
  ok = ok && add(P.prep, prev ? &prev : nullptr, prev ? 1 : 0, &node);
  prev = node;
  ok = ok && add(P.sched, &prev, 1, &node);
  prev = node;
  for (int k = 0; ok && k < P.nf; ++k) {
    if (P.has_pre[k]) {
      ok = add(P.pre[k], &prev, 1, &node);
      prev = node;
    }
    ok = ok && add(P.fam[k], &prev, 1, &node);
    prev = node;
    if (ok && P.has_post[k]) {
      ok = add(P.post[k], &prev, 1, &node);
      prev = node;
    }
  }
  hipGraphExec_t exec = nullptr;
  ok = ok && hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess;
  (void)hipGraphDestroy(g);
  if (!ok) {
    if (exec) (void)hipGraphExecDestroy(exec);
    return RSIM_EDEVICE;
  }
  if (hipGraphLaunch(exec, s) != hipSuccess) {
    (void)hipGraphExecDestroy(exec);
    return RSIM_EDEVICE;
  }
  hipEvent_t ev = nullptr;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess || hipEventRecord(ev, s) != hipSuccess) {
    (void)hipStreamSynchronize(s);
    (void)hipGraphExecDestroy(exec);
    if (ev) (void)hipEventDestroy(ev);
    return RSIM_OK;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  gc_retired(false);
  g_retired.push_back({exec, ev, false});
  if (g_retired.size() > 64) gc_retired(true);
  return RSIM_OK;
}

rsim_status issue(CallPlan& P, hipStream_t s, int use_graph) {
  const rsim_status st = use_graph ? issue_graph(P, s) : issue_eager(P, s);
  if (st != RSIM_OK) return clear_error(st);
  return hipGetLastError() == hipSuccess ? RSIM_OK : RSIM_EDEVICE;
}

// Records the schedule and family kernels of a mix into P.
// The fused front end's features (rsim_simulate_logmel): where they go.
struct FeatOut {
  float* feat = nullptr;
  const int64_t* off = nullptr;
  long long len = 0;
};

void plan_mix(CallPlan& P, const rsim_batch* b, const BatchDev& bd, const TuneDev& td, const float* x,
              const float* h, const float* alpha, float* y, void* ws, int only_fam = -1, size_t cap = 0,
              const FeatOut* fe = nullptr) {
  const DevState& st = dev_state();
  const WsLayout L = layout(b, td, false, st, cap, fe != nullptr);
  char* base = static_cast<char*>(ws);
  SchedArgs SA;
  SA.b = bd;
  SA.tune = td;
  SA.hdr = reinterpret_cast<WsHeader*>(base + L.hdr);
  SA.sched = reinterpret_cast<Sched*>(base + L.sched);
  SA.lists = reinterpret_cast<int*>(base + L.lists);
  SA.costs = reinterpret_cast<float*>(base + L.costs);
  {
    const int cus = st.cus > 0 ? st.cus : 256;
    const long long need = ((long long)b->n_utt + kPrepThreads - 1) / kPrepThreads;
    const long long g = std::max(1LL, std::min(need, (long long)cus * 4));
    P.prep.set(reinterpret_cast<const void*>(&prepare_kernel), dim3((unsigned)g), dim3(kPrepThreads), SA);
  }
  P.sched.set(reinterpret_cast<const void*>(&schedule_kernel), dim3(1), dim3(kSchedThreads), SA);
  bool used[kNumFam];
  families_used(b, td, used);
  P.nf = 0;
  for (int k = 0; k < kNumFam; ++k) {
    const int f = kFamOrder[k];
    if (!used[f] || (only_fam >= 0 && f != only_fam)) continue;
    MixArgs A;
    A.b = bd;
    A.x = x;
    A.h = h;
    A.alpha = alpha;
    A.y = y;
    A.sched = SA.sched;
    A.list = SA.lists;
    A.hdr = SA.hdr;
    A.fam = f;
    A.scratch = reinterpret_cast<cf*>(base + L.fam_scratch[f]);
    A.slot_cf = L.slot_cf[f];
    A.gsplit = L.gsplit[f];
    A.psplit = L.psplit[f];
    A.mmax = kFamMaxM[f];
    A.hspec = L.psplit[f] > 1 ? reinterpret_cast<cf*>(base + L.fam_hspec[f]) : nullptr;
    A.seam = L.psplit[f] > 1 ? reinterpret_cast<float*>(base + L.fam_seam[f]) : nullptr;
    A.feat = fe ? fe->feat : nullptr;
    A.feat_off = fe ? reinterpret_cast<const long long*>(fe->off) : nullptr;
    A.feat_len = fe ? fe->len : 0;
    P.has_pre[P.nf] = P.has_post[P.nf] = L.psplit[f] > 1;
    if (L.psplit[f] > 1) {
      const long long slots = (long long)b->n_utt * b->max_src * b->n_mic;
      const int cus = st.cus > 0 ? st.cus : 256;
      P.pre[P.nf].set(mix_rir_kernel_ptr(f), dim3((unsigned)std::min<long long>(slots, (long long)cus * 2)),
                      dim3(kFamT[f]), A);
      const long long seams = (long long)b->n_utt * L.psplit[f] * b->n_mic;
      P.post[P.nf].set(reinterpret_cast<const void*>(&mix_seam_kernel),
                       dim3((unsigned)std::max<long long>(1, std::min<long long>(seams, (long long)cus * 4))),
                       dim3(kSeamThreads), A);
    }
    P.fam[P.nf++].set(fe ? mix_feat_kernel_ptr(f) : mix_kernel_ptr(f, td.variant[f]), dim3(L.grid[f]),
                      dim3(kFamT[f]), A);
  }
}

// Records the schedule, the zero fill of idle utterances and the adjoint
// family kernels into P.
void plan_bwd(CallPlan& P, const rsim_batch* b, const BatchDev& bd, const TuneDev& td, const float* x,
              const float* h, const float* alpha, const float* gy, float* gx, float* gh, float* galpha,
              void* ws) {
  const DevState& st = dev_state();
  const WsLayout L = layout(b, td, true, st);
  char* base = static_cast<char*>(ws);
  SchedArgs SA;
  SA.b = bd;
  SA.tune = td;
  SA.hdr = reinterpret_cast<WsHeader*>(base + L.hdr);
  SA.sched = reinterpret_cast<Sched*>(base + L.sched);
  SA.lists = reinterpret_cast<int*>(base + L.lists);
  SA.costs = reinterpret_cast<float*>(base + L.costs);
  {
    const int cus = st.cus > 0 ? st.cus : 256;
    const long long need = ((long long)b->n_utt + kPrepThreads - 1) / kPrepThreads;
    const long long g = std::max(1LL, std::min(need, (long long)cus * 4));
    P.prep.set(reinterpret_cast<const void*>(&prepare_kernel), dim3((unsigned)g), dim3(kPrepThreads), SA);
  }
  P.sched.set(reinterpret_cast<const void*>(&schedule_kernel), dim3(1), dim3(kSchedThreads), SA);
  BwdArgs A;
  A.b = bd;
  A.x = x;
  A.h = h;
  A.alpha = alpha;
  A.gy = gy;
  A.gx = gx;
  A.gh = gh;
  A.galpha = galpha;
  A.sched = SA.sched;
  A.list = SA.lists;
  A.hdr = SA.hdr;
  A.fam = -1;
  A.scratch = nullptr;
  A.slot_cf = 0;
  A.nsplit = L.nsplit;
  A.mmax = 0;
  A.partial = nullptr;
  A.hspec = nullptr;
  P.nf = 0;
  const int cus = st.cus > 0 ? st.cus : 256;
  P.fam[P.nf++].set(reinterpret_cast<const void*>(&bwd_zero_kernel), dim3(std::min(b->n_utt, cus * 4)),
                    dim3(256), A);
  bool used[kNumFam];
  families_used(b, td, used);
  for (int k = 0; k < kNumFam; ++k) {
    const int f = kFamOrder[k];
    if (!used[f]) continue;
    A.fam = f;
    A.scratch = reinterpret_cast<cf*>(base + L.fam_scratch[f]);
    A.slot_cf = L.slot_cf[f];
    A.mmax = kFamMaxM[f];
    A.partial = L.nsplit > 1 ? reinterpret_cast<cf*>(base + L.fam_partial[f]) : nullptr;
    A.hspec = L.nsplit > 1 ? reinterpret_cast<cf*>(base + L.fam_hspec[f]) : nullptr;
    if (L.nsplit > 1) {
      P.pre[P.nf].set(bwd_rir_kernel_ptr(f),
                      dim3((unsigned)std::min<long long>((long long)b->n_utt * b->max_src * b->n_mic,
                                                         (long long)cus * 2)),
                      dim3(kFamT[f]), A);
      P.has_pre[P.nf] = true;
    }
    if (L.nsplit > 1) {
      P.post[P.nf].set(bwd_finish_kernel_ptr(f),
                       dim3((unsigned)std::min<long long>((long long)b->n_utt * b->max_src * b->n_mic,
                                                          (long long)cus * 2)),
                       dim3(kFamT[f]), A);
      P.has_post[P.nf] = true;
    }
    P.fam[P.nf++].set(bwd_kernel_ptr(f), dim3(L.grid[f]), dim3(kFamT[f]), A);
  }
}

bool eta_ok(double eta) { return !std::isnan(eta) && eta >= 0.0; }

float cut_scale(double eta) {
  if (std::isinf(eta)) return 0.0f;
  return (float)std::pow(10.0, -eta / 10.0);
}

void plan_truncate(Node& n, const float* h, long long h_len, const int64_t* off, const int32_t* len0,
                   int n_rir, float s, int32_t* n_c, int32_t* len) {
  const DevState& st = dev_state();
  long long grid = (long long)(st.cus > 0 ? st.cus : 256) * 16;
  const long long need = ((long long)n_rir + kTruncWaves - 1) / kTruncWaves;
  if (grid > need) grid = need;
  if (grid < 1) grid = 1;
  TruncArgs A;
  A.h = h;
  A.h_len = h_len;
  A.off = reinterpret_cast<const long long*>(off);
  A.len0 = len0;
  A.n_rir = n_rir;
  A.s = s;
  A.n_c = n_c;
  A.len = len;
  n.set(reinterpret_cast<const void*>(&truncate_kernel), dim3((unsigned)grid), dim3(kTruncThreads), A);
}

int ilog2_exact(int n) {
  if (n <= 0 || (n & (n - 1))) return -1;
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// floor(log2 v) for v >= 1
int ilog2_floor(long long v) {
  int l = 0;
  while ((2LL << l) <= v) ++l;
  return l;
}

rsim_status image_args_ok(int n_rir, int order, double fs, double c0, int max_len, long long h_len) {
  if (n_rir < 0 || order < 0 || order > kImgMaxOrder || !(fs > 0.0) || !(c0 > 0.0) || max_len < 0 || h_len < 0 ||
      !std::isfinite(fs) || !std::isfinite(c0))
    return RSIM_EINVAL;
  if (max_len > kImgMaxLen) return RSIM_EUNSUPPORTED;
  return RSIM_OK;
}

// Persistent workgroups, one per compute unit, taking the RIRs in turn.
void plan_image(Node& n, const double* geom, const double* refl, int n_rir, int order, double fs, double c0, float* h,
                long long h_len, const int64_t* off, const int32_t* len, int max_len) {
  ImageArgs A;
  A.geom = geom;
  A.refl = refl;
  A.h = h;
  A.h_len = h_len;
  A.off = reinterpret_cast<const long long*>(off);
  A.len = len;
  A.n_rir = n_rir;
  A.order = order;
  A.max_len = max_len;
  A.fs = fs;
  A.c0 = c0;
  const DevState& st = dev_state();
  const int cus = st.cus > 0 ? st.cus : 256;
  // one workgroup per CU (its accumulator takes 128 KB of LDS), each taking RIRs in turn
  n.set(reinterpret_cast<const void*>(&image_kernel),
        dim3((unsigned)std::max<long long>(1, std::min<long long>(n_rir, (long long)cus))), dim3(kImgThreads), A);
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

rsim_status rsim_init(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDev) return RSIM_EDEVICE;
  std::lock_guard<std::mutex> lk(g_mu);
  return init_locked(dev);
}

const char* rsim_strerror(rsim_status s) {
  switch (s) {
    case RSIM_OK: return "ok";
    case RSIM_EINVAL: return "invalid argument";
    case RSIM_EWORKSPACE:
      return "workspace missing or too small (rsim_simulate_static: the batch does not fit the static scratch)";
    case RSIM_EUNSUPPORTED: return "unsupported FFT size or hop";
    case RSIM_EDEVICE: return "HIP runtime error";
    case RSIM_ENOTINIT: return "library not initialised on this device (call rsim_init outside capture)";
  }
  return "unknown status";
}

int32_t rsim_version(void) { return 10200; }

rsim_status rsim_truncate_rir(const float* h, int64_t h_len, const int64_t* off, const int32_t* len0,
                              int32_t n_rir, double eta_db, int32_t* n_c, int32_t* len,
                              hipStream_t stream) {
  if (n_rir < 0 || h_len < 0 || !eta_ok(eta_db)) return RSIM_EINVAL;
  if (n_rir == 0) return RSIM_OK;
  if (!arr_ok(h, h_len) || !off || !len0 || !len) return RSIM_EINVAL;
  rsim_status e = ensure_init(stream);
  if (e != RSIM_OK) return e;
  Node n;
  plan_truncate(n, h, h_len, off, len0, n_rir, cut_scale(eta_db), n_c, len);
  if (hipLaunchKernel(n.fn, n.grid, n.block, n.p(), 0, stream) != hipSuccess) return clear_error(RSIM_EDEVICE);
  return RSIM_OK;
}

size_t rsim_mix_workspace_bytes(const rsim_batch* b, const rsim_tune* tune, int32_t backward) {
  if (!batch_ok(b) || !tune_ok(tune)) return 0;
  (void)ensure_init(nullptr);  // launch geometry of this device, when there is one
  const TuneDev td = to_dev(tune);
  return layout(b, td, backward != 0, dev_state()).total;
}

rsim_status rsim_mix(const rsim_batch* b, const float* x, const float* h, const float* alpha, float* y,
                     void* ws, size_t ws_bytes, const rsim_tune* tune, int32_t use_graph,
                     hipStream_t stream) {
  if (!batch_ok(b) || !tune_ok(tune)) return RSIM_EINVAL;
  if (b->n_utt == 0) return RSIM_OK;
  if (!arr_ok(x, b->x_len) || !arr_ok(h, b->h_len) || !alpha || !arr_ok(y, b->y_len)) return RSIM_EINVAL;
  const rsim_status e = ensure_init(stream);
  const TuneDev td = to_dev(tune);
  const WsLayout L = layout(b, td, false, dev_state());
  if (!ws || ws_bytes < L.total) return RSIM_EWORKSPACE;
  if (e != RSIM_OK) return e;
  const BatchDev bd = to_dev(b);
  CallPlan P;
  plan_mix(P, b, bd, td, x, h, alpha, y, ws);
  return issue(P, stream, use_graph);
}

rsim_status rsim_simulate(const rsim_batch* b, const float* x, const float* h, const float* alpha,
                          double eta_db, int32_t* rir_len_out, float* y, void* ws, size_t ws_bytes,
                          const rsim_tune* tune, int32_t use_graph, hipStream_t stream) {
  if (!b || !eta_ok(eta_db) || !rir_len_out || !tune_ok(tune)) return RSIM_EINVAL;
  rsim_batch bb = *b;
  bb.rir_len = rir_len_out;
  if (!batch_ok(&bb)) return RSIM_EINVAL;
  if (bb.n_utt == 0) return RSIM_OK;
  if (!arr_ok(x, bb.x_len) || !arr_ok(h, bb.h_len) || !alpha || !arr_ok(y, bb.y_len)) return RSIM_EINVAL;
  const rsim_status e = ensure_init(stream);
  const TuneDev td = to_dev(tune);
  const WsLayout L = layout(&bb, td, false, dev_state());
  if (!ws || ws_bytes < L.total) return RSIM_EWORKSPACE;
  if (e != RSIM_OK) return e;
  const long long n_rir = (long long)bb.n_utt * bb.max_src * bb.n_mic;
  if (n_rir > 0x7fffffffLL) return RSIM_EINVAL;
  const BatchDev bd = to_dev(&bb);
  const float s = cut_scale(eta_db);
  CallPlan P;
  P.has_cut = true;
  plan_truncate(P.cut, h, bb.h_len, bb.rir_off, bb.rir_len0, (int)n_rir, s, nullptr, rir_len_out);
  plan_mix(P, &bb, bd, td, x, h, alpha, y, ws);
  return issue(P, stream, use_graph);
}

rsim_status rsim_simulate_static(const rsim_batch* b, const float* x, const float* h, const float* alpha,
                                 double eta_db, int32_t* rir_len_out, float* y, const rsim_tune* tune,
                                 hipStream_t stream) {
  if (!b || !eta_ok(eta_db) || !rir_len_out || !tune_ok(tune)) return RSIM_EINVAL;
  rsim_batch bb = *b;
  bb.rir_len = rir_len_out;
  if (!batch_ok(&bb)) return RSIM_EINVAL;
  if (bb.n_utt == 0) return RSIM_OK;
  if (!arr_ok(x, bb.x_len) || !arr_ok(h, bb.h_len) || !alpha || !arr_ok(y, bb.y_len)) return RSIM_EINVAL;
  const long long n_rir = (long long)bb.n_utt * bb.max_src * bb.n_mic;
  if (n_rir > 0x7fffffffLL) return RSIM_EINVAL;
  const rsim_status e = ensure_init(stream);
  if (e != RSIM_OK) return e;
  const DevState& st = dev_state();
  if (!st.static_ws) return RSIM_EDEVICE;
  const TuneDev td = to_dev(tune);
  const size_t cap = RSIM_STATIC_SCRATCH_BYTES;
  if (layout(&bb, td, false, st, cap).total > cap) return RSIM_EWORKSPACE;
  const BatchDev bd = to_dev(&bb);
  CallPlan P;
  P.has_cut = true;
  plan_truncate(P.cut, h, bb.h_len, bb.rir_off, bb.rir_len0, (int)n_rir, cut_scale(eta_db), nullptr, rir_len_out);
  plan_mix(P, &bb, bd, td, x, h, alpha, y, st.static_ws, -1, cap);
  return issue(P, stream, 0);
}

size_t rsim_simulate_logmel_workspace_bytes(const rsim_batch* b, const rsim_tune* tune) {
  if (!batch_ok(b) || !tune_ok(tune)) return 0;
  (void)ensure_init(nullptr);
  return layout(b, feat_tune(tune), false, dev_state(), 0, true).total;
}

rsim_status rsim_simulate_logmel(const rsim_batch* b, const float* x, const float* h, const float* alpha,
                                 double eta_db, int32_t* rir_len_out, float* feat, const int64_t* feat_off,
                                 int64_t feat_len, void* ws, size_t ws_bytes, const rsim_tune* tune,
                                 int32_t use_graph, hipStream_t stream) {
  if (!b || !eta_ok(eta_db) || !rir_len_out || !tune_ok(tune) || feat_len < 0) return RSIM_EINVAL;
  rsim_batch bb = *b;
  bb.rir_len = rir_len_out;
  if (!batch_ok(&bb)) return RSIM_EINVAL;
  if (bb.n_utt == 0) return RSIM_OK;
  if (!arr_ok(x, bb.x_len) || !arr_ok(h, bb.h_len) || !alpha || !feat || !feat_off) return RSIM_EINVAL;
  if (bb.n_mic > kFeatMics) return RSIM_EUNSUPPORTED;
  if (bb.fft_log2n && (bb.fft_sizes == 0 || (bb.fft_sizes & ~kFeatSizeBits))) return RSIM_EUNSUPPORTED;
  const long long n_rir = (long long)bb.n_utt * bb.max_src * bb.n_mic;
  if (n_rir > 0x7fffffffLL) return RSIM_EINVAL;
  const rsim_status e = ensure_init(stream);
  const TuneDev td = feat_tune(tune);
  const WsLayout L = layout(&bb, td, false, dev_state(), 0, true);
  if (!ws || ws_bytes < L.total) return RSIM_EWORKSPACE;
  if (e != RSIM_OK) return e;
  const BatchDev bd = to_dev(&bb);
  CallPlan P;
  P.has_cut = true;
  plan_truncate(P.cut, h, bb.h_len, bb.rir_off, bb.rir_len0, (int)n_rir, cut_scale(eta_db), nullptr, rir_len_out);
  FeatOut fe;
  fe.feat = feat;
  fe.off = feat_off;
  fe.len = feat_len;
  plan_mix(P, &bb, bd, td, x, h, alpha, nullptr, ws, -1, 0, &fe);
  return issue(P, stream, use_graph);
}

size_t rsim_ola_workspace_bytes(int32_t fft_n) {
  const int l2 = ilog2_exact(fft_n);
  if (l2 < 9 || l2 > 15) return 0;
  rsim_batch b;
  std::memset(&b, 0, sizeof(b));
  b.n_utt = 1;
  b.n_mic = 1;
  b.max_src = 1;
  int32_t dummy = 0;
  b.fft_log2n = &dummy;  // marks a forced size
  b.fft_sizes = 1 << l2;
  (void)ensure_init(nullptr);
  return align256(sizeof(OlaDesc)) + layout(&b, default_tune(), false, dev_state()).total;
}

rsim_status rsim_ola_convolve(const float* x, int32_t nx, const float* h, int32_t nh, int32_t fft_n,
                              int32_t hop, float* y, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!x || !h || !y || nx < 1 || nh < 1 || hop < 0) return RSIM_EINVAL;
  const int l2 = ilog2_exact(fft_n);
  if (l2 < 9 || l2 > 15) return RSIM_EUNSUPPORTED;
  if (hop == 0) hop = fft_n - nh + 1;
  if (hop < 1 || (long long)hop + nh - 1 > fft_n) return RSIM_EUNSUPPORTED;
  if ((long long)nx + nh - 1 > 0x7fffffffLL) return RSIM_EINVAL;
  const size_t need = rsim_ola_workspace_bytes(fft_n);
  if (!ws || ws_bytes < need) return RSIM_EWORKSPACE;
  rsim_status e = ensure_init(stream);
  if (e != RSIM_OK) return e;
  char* base = static_cast<char*>(ws);
  OlaDesc* d = reinterpret_cast<OlaDesc*>(base);
  hipLaunchKernelGGL(ola_setup_kernel, dim3(1), dim3(1), 0, stream, d, nx, nh, l2, hop);
  rsim_batch b;
  std::memset(&b, 0, sizeof(b));
  b.n_utt = 1;
  b.n_mic = 1;
  b.max_src = 1;
  b.max_rir_len0 = nh;
  b.x_len = nx;
  b.h_len = nh;
  b.y_len = (int64_t)nx + nh - 1;
  b.n_src = &d->n_src;
  b.src_len = &d->src_len;
  b.src_off = reinterpret_cast<const int64_t*>(&d->src_off);
  b.rir_off = reinterpret_cast<const int64_t*>(&d->rir_off);
  b.rir_len0 = &d->rir_len0;
  b.rir_len = &d->rir_len;
  b.out_off = reinterpret_cast<const int64_t*>(&d->out_off);
  b.out_stride = &d->out_stride;
  b.out_len = &d->out_len;
  b.order = nullptr;
  b.fft_log2n = &d->log2n;
  b.fft_sizes = 1 << l2;
  b.hop = &d->hop;
  const TuneDev td = default_tune();
  const BatchDev bd = to_dev(&b);
  CallPlan P;
  plan_mix(P, &b, bd, td, x, h, &d->alpha, y, base + align256(sizeof(OlaDesc)), family_of_log2n(l2));
  return issue(P, stream, 0);
}

rsim_status rsim_mix_backward(const rsim_batch* b, const float* x, const float* h, const float* alpha,
                              const float* grad_y, float* grad_x, float* grad_h, float* grad_alpha,
                              void* ws, size_t ws_bytes, const rsim_tune* tune, hipStream_t stream) {
  if (!batch_ok(b) || !tune_ok(tune)) return RSIM_EINVAL;
  if (b->n_utt == 0) return RSIM_OK;
  if (!arr_ok(x, b->x_len) || !arr_ok(h, b->h_len) || !alpha || !arr_ok(grad_y, b->y_len) ||
      !arr_ok(grad_x, b->x_len) || !arr_ok(grad_h, b->h_len))
    return RSIM_EINVAL;
  const rsim_status e = ensure_init(stream);
  const TuneDev td = to_dev(tune);
  const WsLayout L = layout(b, td, true, dev_state());
  if (!ws || ws_bytes < L.total) return RSIM_EWORKSPACE;
  if (e != RSIM_OK) return e;
  const BatchDev bd = to_dev(b);
  CallPlan P;
  plan_bwd(P, b, bd, td, x, h, alpha, grad_y, grad_x, grad_h, grad_alpha, ws);
  return issue(P, stream, 0);
}

rsim_status rsim_source_power(const rsim_batch* b, const float* x, double* power, hipStream_t stream) {
  if (!batch_ok(b)) return RSIM_EINVAL;
  if (b->n_utt == 0) return RSIM_OK;
  if (!arr_ok(x, b->x_len) || !power) return RSIM_EINVAL;
  rsim_status e = ensure_init(stream);
  if (e != RSIM_OK) return e;
  const long long slots = (long long)b->n_utt * b->max_src;
  int grid = dev_state().cus * 8;
  if (grid > slots) grid = (int)slots;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(power_kernel, dim3(grid), dim3(256), 0, stream, to_dev(b), x, power);
  return hipGetLastError() == hipSuccess ? RSIM_OK : RSIM_EDEVICE;
}

rsim_status rsim_snr_gains(const double* p_dry, const double* snr_db, int32_t I, int32_t J,
                           float* alpha) {
  if (I < 0 || J < 1) return RSIM_EINVAL;
  if (I == 0) return RSIM_OK;
  if (!p_dry || !snr_db || !alpha) return RSIM_EINVAL;
  for (int j = 0; j < J; ++j) alpha[j] = 1.0f;
  const double p0 = p_dry[0];
  for (int i = 1; i < I; ++i) {
    const double pi = p_dry[i];
    const double a = pi <= 0.0 ? 0.0 : std::sqrt(p0 / (pi * std::pow(10.0, snr_db[i] / 10.0)));
    for (int j = 0; j < J; ++j) alpha[i * J + j] = (float)a;
  }
  return RSIM_OK;
}

rsim_status rsim_device_status(hipStream_t stream, int32_t* status) {
  if (!status) return RSIM_EINVAL;
  rsim_status e = ensure_init(stream);
  if (e != RSIM_OK) return e;
  int v = 0;
  const int zero = 0;
  if (hipMemcpyFromSymbolAsync(&v, HIP_SYMBOL(g_status), sizeof(int), 0, hipMemcpyDeviceToHost, stream) !=
          hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return clear_error(RSIM_EDEVICE);
  if (hipMemcpyToSymbolAsync(HIP_SYMBOL(g_status), &zero, sizeof(int), 0, hipMemcpyHostToDevice, stream) !=
          hipSuccess ||
      hipStreamSynchronize(stream) != hipSuccess)
    return clear_error(RSIM_EDEVICE);
  *status = v;
  return RSIM_OK;
}

rsim_status rsim_image_rir(const double* geom, const double* refl, int32_t n_rir, int32_t order, double fs,
                           double c0, float* h, int64_t h_len, const int64_t* off, const int32_t* len,
                           int32_t max_len, hipStream_t stream) {
  const rsim_status v = image_args_ok(n_rir, order, fs, c0, max_len, h_len);
  if (v != RSIM_OK) return v;
  if (n_rir == 0 || max_len == 0) return RSIM_OK;
  if (!geom || !refl || !h || !off || !len) return RSIM_EINVAL;
  const rsim_status e = ensure_init(stream);
  if (e != RSIM_OK) return e;
  Node n;
  plan_image(n, geom, refl, n_rir, order, fs, c0, h, h_len, off, len, max_len);
  if (hipLaunchKernel(n.fn, n.grid, n.block, n.p(), 0, stream) != hipSuccess) return clear_error(RSIM_EDEVICE);
  return RSIM_OK;
}

rsim_status rsim_simulate_rooms(const rsim_batch* b, const float* x, float* h, const double* geom,
                                const double* refl, int32_t order, double fs, double c0, const float* alpha,
                                double eta_db, int32_t* rir_len_out, float* y, void* ws, size_t ws_bytes,
                                const rsim_tune* tune, int32_t use_graph, hipStream_t stream) {
  if (!b || !eta_ok(eta_db) || !rir_len_out || !tune_ok(tune)) return RSIM_EINVAL;
  rsim_batch bb = *b;
  bb.rir_len = rir_len_out;
  if (!batch_ok(&bb)) return RSIM_EINVAL;
  const long long n_rir = (long long)bb.n_utt * bb.max_src * bb.n_mic;
  if (n_rir > 0x7fffffffLL) return RSIM_EINVAL;
  const rsim_status v = image_args_ok((int)n_rir, order, fs, c0, bb.max_rir_len0, bb.h_len);
  if (v != RSIM_OK) return v;
  if (bb.n_utt == 0) return RSIM_OK;
  if (!arr_ok(x, bb.x_len) || !arr_ok(h, bb.h_len) || !geom || !refl || !alpha || !arr_ok(y, bb.y_len))
    return RSIM_EINVAL;
  const rsim_status e = ensure_init(stream);
  const TuneDev td = to_dev(tune);
  const WsLayout L = layout(&bb, td, false, dev_state());
  if (!ws || ws_bytes < L.total) return RSIM_EWORKSPACE;
  if (e != RSIM_OK) return e;
  const BatchDev bd = to_dev(&bb);
  CallPlan P;
  P.has_gen = bb.max_rir_len0 > 0;
  if (P.has_gen)
    plan_image(P.gen, geom, refl, (int)n_rir, order, fs, c0, h, bb.h_len, bb.rir_off, bb.rir_len0,
               bb.max_rir_len0);
  P.has_cut = true;
  plan_truncate(P.cut, h, bb.h_len, bb.rir_off, bb.rir_len0, (int)n_rir, cut_scale(eta_db), nullptr, rir_len_out);
  plan_mix(P, &bb, bd, td, x, h, alpha, y, ws);
  return issue(P, stream, use_graph);
}

rsim_status rsim_reverb_energy(const rsim_batch* b, const float* x, const float* h, double* energy,
                               hipStream_t stream) {
  if (!batch_ok(b)) return RSIM_EINVAL;
  if (b->n_utt == 0) return RSIM_OK;
  if (!arr_ok(x, b->x_len) || !arr_ok(h, b->h_len) || !energy) return RSIM_EINVAL;
  const rsim_status e = ensure_init(stream);
  if (e != RSIM_OK) return e;
  const BatchDev bd = to_dev(b);
  const DevState& st = dev_state();
  const int cus = st.cus > 0 ? st.cus : 256;
  const long long items = (long long)b->n_utt * b->max_src;
  // transforms of 2^14 and 2^15 points only (energy_log2n)
  for (int f : {family_of_log2n(14), family_of_log2n(15)}) {
    EnergyArgs A;
    A.b = bd;
    A.x = x;
    A.h = h;
    A.energy = energy;
    A.fam = f;
    void* args[] = {&A};
    // one workgroup per CU (the exchange buffers take most of its LDS), each
    // with a balanced range of the family's slots
    const unsigned grid = (unsigned)std::max<long long>(1, std::min<long long>(items, (long long)cus));
    if (hipLaunchKernel(energy_kernel_ptr(f), dim3(grid), dim3(kFamT[f]), args, 0, stream) != hipSuccess)
      return clear_error(RSIM_EDEVICE);
  }
  return RSIM_OK;
}

rsim_status rsim_snr_gains_reverb(const double* energy, const double* snr_db, int32_t I, int32_t J, float* alpha) {
  if (I < 0 || J < 1 || (I > 0 && (!energy || !snr_db || !alpha))) return RSIM_EINVAL;
  for (int i = 0; i < I; ++i)
    for (int j = 0; j < J; ++j) {
      double a = 1.0;
      if (i > 0) {
        const double e0 = energy[j], ei = energy[i * J + j];
        a = (ei > 0.0 && e0 > 0.0) ? std::sqrt(e0 / (ei * std::pow(10.0, snr_db[i] / 10.0))) : 0.0;
      }
      alpha[i * J + j] = (float)a;
    }
  return RSIM_OK;
}

rsim_status rsim_logmel(const rsim_batch* b, const float* y, float* feat, const int64_t* feat_off, int64_t feat_len,
                        int32_t max_frames, hipStream_t stream) {
  if (!batch_ok(b) || max_frames < 0 || feat_len < 0) return RSIM_EINVAL;
  if (b->n_utt == 0 || max_frames == 0) return RSIM_OK;
  if (!arr_ok(y, b->y_len) || !feat || !feat_off) return RSIM_EINVAL;
  const rsim_status e = ensure_init(stream);
  if (e != RSIM_OK) return e;
  MelArgs A;
  A.b = to_dev(b);
  A.y = y;
  A.feat = feat;
  A.feat_off = reinterpret_cast<const long long*>(feat_off);
  A.feat_len = feat_len;
  A.chunks = (max_frames + kMelGroups - 1) / kMelGroups;
  const DevState& st = dev_state();
  const int cus = st.cus > 0 ? st.cus : 256;
  const long long items = (long long)b->n_utt * b->n_mic * A.chunks;
  const unsigned grid = (unsigned)std::max<long long>(1, std::min<long long>(items, (long long)cus * 16));
  hipLaunchKernelGGL(logmel_kernel, dim3(grid), dim3(kMelGroups * 32), 0, stream, A);
  return hipGetLastError() == hipSuccess ? RSIM_OK : clear_error(RSIM_EDEVICE);
}

rsim_status rsim_fft_filter_sizes(const int32_t* src_len, const int32_t* rir_len0, int32_t n_utt, int32_t max_src,
                                  int32_t n_mic, int32_t* log2n) {
  if (n_utt < 0 || max_src < 1 || n_mic < 1) return RSIM_EINVAL;
  if (n_utt == 0) return RSIM_OK;
  if (!src_len || !rir_len0 || !log2n) return RSIM_EINVAL;
  const long long per = (long long)max_src * n_mic;
  for (int u = 0; u < n_utt; ++u) {
    int l0 = 0;
    for (long long k = 0; k < per; ++k) l0 = std::max(l0, rir_len0[u * per + k]);
    const long long need = (long long)src_len[u] + l0 - 1;
    if (src_len[u] <= 0 || l0 <= 0) {
      log2n[u] = 0;
      continue;
    }
    int m = 1;
    while ((1LL << m) < need) ++m;
    log2n[u] = m;
  }
  return RSIM_OK;
}

size_t rsim_fft_filter_workspace_bytes(const rsim_batch* b, int32_t fft_log2n, int32_t chunk) {
  if (!batch_ok(b) || fft_log2n < 1 || fft_log2n > 20 || chunk < 1) return 0;
  const size_t N = (size_t)1 << fft_log2n, C = (size_t)chunk, S = (size_t)b->max_src;
  return 3 * S * C * N * sizeof(cf);
}

rsim_status rsim_fft_filter(const rsim_batch* b, const float* x, const float* h, const float* alpha, float* y,
                            int32_t fft_log2n, int32_t chunk, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (!batch_ok(b) || fft_log2n < 1 || fft_log2n > 20 || chunk < 1) return RSIM_EINVAL;
  if (b->n_utt == 0) return RSIM_OK;
  if (!arr_ok(x, b->x_len) || !arr_ok(h, b->h_len) || !alpha || !arr_ok(y, b->y_len)) return RSIM_EINVAL;
  const size_t need = rsim_fft_filter_workspace_bytes(b, fft_log2n, chunk);
  if (!ws || ws_bytes < need) return RSIM_EWORKSPACE;
  const rsim_status e = ensure_init(stream);
  if (e != RSIM_OK) return e;
  const long long N = 1LL << fft_log2n, C = chunk, S = b->max_src;
  cf* X = static_cast<cf*>(ws);  // [C][S][N] source spectra
  cf* H = X + C * S * N;         // [C][S][N] RIR spectra of one mic
  cf* tmp = H + C * S * N;       // [C][S][N] between the two steps
  const DevState& st = dev_state();
  const int cus = st.cus > 0 ? st.cus : 256;
  // N = N1 N2, N1 = 2^l1 >= N2 = 2^l2, both at most 1024 points
  const int l1 = (fft_log2n + 1) / 2, l2 = fft_log2n / 2;
  FfStep base{};
  base.sig_len = N;
  base.log2n = fft_log2n;
  base.b = to_dev(b);
  base.x = x;
  base.h = h;
  base.alpha = alpha;
  base.y = y;
  base.X = X;
  base.H = H;
  base.S = (int)S;
  // step A (first) or B of `count` transforms from `in` to `out`
  auto step = [&](FfStep S_, const cf* in, cf* out, int count, bool inv, bool first) {
    S_.in = in;
    S_.out = out;
    S_.count = count;
    if (first) {  // step A: N2 sequences of N1 points (stride N2), twiddled
      S_.log2l = l1;
      S_.cols = 1 << l2;
      S_.in_cs = 1;
      S_.in_ns = 1LL << l2;
      S_.out_cs = 1;
      S_.out_ks = 1LL << l2;
      S_.n_fast = 0;
      S_.twiddle = 1;
    } else {  // step B: N1 rows of N2 points, outputs at k1 + N1 k2
      S_.log2l = l2;
      S_.cols = 1 << l1;
      S_.in_cs = 1LL << l2;
      S_.in_ns = 1;
      S_.out_cs = 1;
      S_.out_ks = 1LL << l1;
      S_.n_fast = 1;
      S_.twiddle = 0;
    }
    S_.log2c = std::min(ilog2_floor(kFfTile) - S_.log2l, ilog2_floor(S_.cols));
    const long long items = (long long)count * (S_.cols >> S_.log2c);
    const dim3 grid((unsigned)std::max<long long>(1, std::min<long long>(items, (long long)cus * 2)));
    void* args[] = {&S_};
    const void* fn = inv ? reinterpret_cast<const void*>(&ff_step_kernel<true>)
                         : reinterpret_cast<const void*>(&ff_step_kernel<false>);
    return hipLaunchKernel(fn, grid, dim3(kFfStepThreads), args, 0, stream) == hipSuccess;
  };
  for (int u0 = 0; u0 < b->n_utt; u0 += chunk) {
    const int nu = std::min(chunk, b->n_utt - u0);
    const int cs = (int)(nu * S);
    FfStep F = base;
    F.u0 = u0;
    F.n_src = b->n_src;  // forward transforms run over source slots
    // the sources' spectra: real samples -> A -> tmp -> B -> X
    FfStep A1 = F, B1 = F;
    A1.in_kind = 1;
    if (!step(A1, nullptr, tmp, cs, false, true) || !step(B1, tmp, X, cs, false, false))
      return clear_error(RSIM_EDEVICE);
    for (int j = 0; j < b->n_mic; ++j) {
      // the cut RIRs' spectra of mic j -> H
      FfStep A2 = F, B2 = F;
      A2.in_kind = 2;
      A2.j = j;
      if (!step(A2, nullptr, tmp, cs, false, true) || !step(B2, tmp, H, cs, false, false))
        return clear_error(RSIM_EDEVICE);
      // one inverse per utterance of sum_i alpha H X, stored as y_j
      FfStep A3 = base, B3 = base;
      A3.u0 = B3.u0 = u0;
      A3.in_kind = 3;
      A3.j = B3.j = j;
      B3.out_kind = 1;
      if (!step(A3, nullptr, tmp, nu, true, true) || !step(B3, tmp, nullptr, nu, true, false))
        return clear_error(RSIM_EDEVICE);
    }
  }
  return hipGetLastError() == hipSuccess ? RSIM_OK : clear_error(RSIM_EDEVICE);
}

rsim_status rsim_rfft(const float* x, int32_t n, int32_t count, float* spec, hipStream_t stream) {
  const int l2 = ilog2_exact(n);
  if (l2 < 9 || l2 > 15) return RSIM_EUNSUPPORTED;
  if (count < 0 || (count > 0 && (!x || !spec))) return RSIM_EINVAL;
  if (count == 0) return RSIM_OK;
  rsim_status e = ensure_init(stream);
  if (e != RSIM_OK) return e;
  sfor<kNumSizes>([&](auto c) {
    constexpr int L2 = kMinL2 + decltype(c)::value;
    using PL = PlanOf<L2>;
    if (l2 == L2) hipLaunchKernelGGL(rfft_kernel<PL>, dim3(count), dim3(PL::T), 0, stream, x, spec);
  });
  return hipGetLastError() == hipSuccess ? RSIM_OK : RSIM_EDEVICE;
}

rsim_status rsim_irfft(const float* spec, int32_t n, int32_t count, float* x, hipStream_t stream) {
  const int l2 = ilog2_exact(n);
  if (l2 < 9 || l2 > 15) return RSIM_EUNSUPPORTED;
  if (count < 0 || (count > 0 && (!x || !spec))) return RSIM_EINVAL;
  if (count == 0) return RSIM_OK;
  rsim_status e = ensure_init(stream);
  if (e != RSIM_OK) return e;
  sfor<kNumSizes>([&](auto c) {
    constexpr int L2 = kMinL2 + decltype(c)::value;
    using PL = PlanOf<L2>;
    if (l2 == L2) hipLaunchKernelGGL(irfft_kernel<PL>, dim3(count), dim3(PL::T), 0, stream, spec, x);
  });
  return hipGetLastError() == hipSuccess ? RSIM_OK : RSIM_EDEVICE;
}

}  // extern "C"

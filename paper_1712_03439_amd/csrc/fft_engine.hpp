// Register/LDS real-FFT engine for gfx950 (CDNA4), one transform per workgroup.
//
// The block filtering of Sec. 2.2 (eqs. 4-6) needs, per block, a real FFT of
// size N = 2M, a product over the half spectrum 0 <= k <= N/2 (real signals
// have a Hermitian spectrum, Sec. 2.2 before eq. 5) and an inverse real FFT.
// Here a real block x[0..N) is packed as z[n] = x[2n] + i x[2n+1] (M complex
// points) and transformed by a Stockham mixed-radix FFT whose passes run in
// registers (P = M/T points per thread) with one LDS exchange between passes.
//
// Layout conventions (T threads, thread t):
//  * time domain: v[r] = z[t + r T], r < P  (coalesced global loads/stores)
//  * frequency domain ("slot layout"): the last pass has radix R = P/2 and each
//    thread owns two of its butterflies, ja = t and jb = 2T - t (thread 0: 0
//    and T).  Slot q < R holds bin ja + 2Tq, slot R + q holds bin jb + 2Tq.
//    Bins k and M - k therefore always live in the same thread, so the real
//    post/pre-processing is register-local.  After post(), thread 0's slots
//    are permuted (see perm_t0) and its slot SP packs the two real bins
//    X[0] (x) and X[N/2] (y).
//  * Spectra kept in memory use index (slot * T + t): coalesced per slot.
//
// Scaling: forward() + post() gives 2 X[k]; pre() + inverse() of 2 Y gives
// 4 M y.  A product 2X * (c 2H) with c = 1/(8M) therefore returns h * x.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

namespace rsim {

typedef float2 cf;

__device__ __forceinline__ cf mk(float x, float y) { return make_float2(x, y); }
__device__ __forceinline__ cf operator+(cf a, cf b) { return mk(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ cf operator-(cf a, cf b) { return mk(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ cf operator-(cf a) { return mk(-a.x, -a.y); }
// a * w
__device__ __forceinline__ cf cmul(cf a, cf w) {
  return mk(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}
// a * conj(w)
__device__ __forceinline__ cf cmulc(cf a, cf w) {
  return mk(a.x * w.x + a.y * w.y, a.y * w.x - a.x * w.y);
}
__device__ __forceinline__ cf conjf2(cf a) { return mk(a.x, -a.y); }

// Hides a pointer's value from the optimiser so that table loads made through
// it are not hoisted out of the caller's loops (which would keep every
// twiddle of every pass live in registers for the whole kernel).
template <class T>
__device__ __forceinline__ const T* opaque(const T* p) {
  asm volatile("" : "+s"(p));
  return p;
}
// ------------------------------------------------------------ buffer access
// Raw buffer resources: the base lives in scalar registers and each access
// needs one 32-bit lane offset.  The `vo` operand (and any immediate the
// compiler folds out of it) is range-checked against the resource size:
// loads past it return 0 and stores past it are dropped, which gives the
// zero padding of a signal block and the clipping of an output block without
// branches.  The `so` operand is not range-checked (constant strides only).
// The check is per 32-bit word: a 64-bit access that straddles the end keeps
// its first word and drops (reads 0 for) the second.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data format (gfx9 family)

__device__ __forceinline__ rsrc_t make_rsrc(const void* p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, bytes, kRsrcWord3);
}
__device__ __forceinline__ float ld1(rsrc_t r, int vo, int so = 0) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
}
__device__ __forceinline__ void st1(rsrc_t r, int vo, float v, int so = 0) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, so, 0);
}
__device__ __forceinline__ cf ld2(rsrc_t r, int vo, int so = 0) {
  return __builtin_bit_cast(cf, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
}
typedef float f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f4 ld4(rsrc_t r, int vo, int so = 0) {
  return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0));
}
__device__ __forceinline__ void st2(rsrc_t r, int vo, cf v, int so = 0) {
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, vo, so, 0);
}

// Same for the thread index: values derived from it inside a helper (LDS and
// global offsets) are recomputed per call instead of being hoisted out of the
// caller's loops and kept live (or spilled) for the whole kernel.
__device__ __forceinline__ int opaque_v(int x) {
  asm volatile("" : "+v"(x));
  return x;
}
__device__ __forceinline__ cf opaque_c(cf z) {
  asm volatile("" : "+v"(z.x), "+v"(z.y));
  return z;
}
// a * a
__device__ __forceinline__ cf csq(cf a) {
  return mk(__builtin_fmaf(a.x, a.x, -(a.y * a.y)), 2.f * (a.x * a.y));
}
// acc + a * b
__device__ __forceinline__ cf cmac(cf acc, cf a, cf b) {
  return mk(__builtin_fmaf(a.x, b.x, __builtin_fmaf(-a.y, b.y, acc.x)),
            __builtin_fmaf(a.x, b.y, __builtin_fmaf(a.y, b.x, acc.y)));
}
// acc + conj(a) * b
__device__ __forceinline__ cf cmacc(cf acc, cf a, cf b) {
  return mk(__builtin_fmaf(a.x, b.x, __builtin_fmaf(a.y, b.y, acc.x)),
            __builtin_fmaf(a.x, b.y, __builtin_fmaf(-a.y, b.x, acc.y)));
}

// ------------------------------------------------------------ compile-time loops
template <class F, int... Is>
__host__ __device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, Is...>) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__host__ __device__ __forceinline__ void sfor(F&& f) {
  sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// ------------------------------------------------ multiplication by exp(-2 pi i m/32)
// cos(2 pi m / 32) for m = 0..8.
constexpr float kC32[9] = {1.0f,
                           0.980785280403230449126182236134239f,
                           0.923879532511286756128183189396788f,
                           0.831469612302545237078788377617906f,
                           0.707106781186547524400844362104849f,
                           0.555570233019602224742830813948533f,
                           0.382683432365089771728459984030399f,
                           0.195090322016128267848284868477022f,
                           0.0f};
constexpr float cos32(int m) {
  m = ((m % 32) + 32) % 32;
  return m <= 8 ? kC32[m] : m <= 16 ? -kC32[16 - m] : m <= 24 ? -kC32[m - 16] : kC32[32 - m];
}
constexpr float sin32(int m) { return cos32(m - 8); }

// a * exp(-2 pi i m / 32), with the multiplications that are sign flips or
// swaps done exactly.
template <int M32>
__device__ __forceinline__ cf rot32(cf a) {
  constexpr int m = ((M32 % 32) + 32) % 32;
  constexpr float h = kC32[4];
  if constexpr (m == 0) {
    return a;
  } else if constexpr (m == 8) {  // -i
    return mk(a.y, -a.x);
  } else if constexpr (m == 16) {
    return mk(-a.x, -a.y);
  } else if constexpr (m == 24) {  // +i
    return mk(-a.y, a.x);
  } else if constexpr (m == 4) {
    return mk((a.x + a.y) * h, (a.y - a.x) * h);
  } else if constexpr (m == 12) {
    return mk((a.y - a.x) * h, -(a.x + a.y) * h);
  } else if constexpr (m == 20) {
    return mk(-(a.x + a.y) * h, (a.x - a.y) * h);
  } else if constexpr (m == 28) {
    return mk((a.x - a.y) * h, (a.x + a.y) * h);
  } else {
    constexpr float c = cos32(m), s = sin32(m);
    // (a.x + i a.y)(c - i s)
    return mk(__builtin_fmaf(a.x, c, a.y * s), __builtin_fmaf(a.y, c, -(a.x * s)));
  }
}

// a * W_R^K with W_R = exp(-2 pi i / R) (forward) or its conjugate (inverse).
template <int R, int K, bool INV>
__device__ __forceinline__ cf twc(cf a) {
  static_assert(32 % R == 0, "radix must divide 32");
  return rot32<(INV ? -K : K) * (32 / R)>(a);
}

// Calls f(r, w^r) for r = 1..R-1 (r as a compile-time constant), forming the
// powers on the fly from w, w^2, w^3, w^4 and the anchors w^{4m}: at most
// about R/4 + 2 roundings per power and a handful of live registers.
template <int R, class F>
__device__ __forceinline__ void for_powers(cf w1, F&& f) {
  const cf w2 = csq(w1);
  const cf w3 = cmul(w2, w1);
  const cf w4 = csq(w2);
  cf g = w4;
  sfor<R - 1>([&](auto rc) {
    constexpr int r = decltype(rc)::value + 1;
    constexpr int e = r % 4;
    if constexpr (r < 4) {
      f(std::integral_constant<int, r>{}, e == 1 ? w1 : e == 2 ? w2 : w3);
    } else if constexpr (e == 0) {
      if constexpr (r > 4) g = cmul(g, w4);
      f(std::integral_constant<int, r>{}, g);
    } else {
      f(std::integral_constant<int, r>{}, cmul(g, e == 1 ? w1 : e == 2 ? w2 : w3));
    }
  });
}

// --------------------------------------------------------------- DFT codelets
// In-place R-point DFT of v[0..R) (natural order in and out); INV uses the
// conjugate roots (no 1/R scaling).
template <int R, bool INV>
__device__ __forceinline__ void dft(cf* v);

template <bool INV>
__device__ __forceinline__ void radix4(cf& a, cf& b, cf& c, cf& d) {
  cf t0 = a + c, t1 = a - c, t2 = b + d, t3 = b - d;
  a = t0 + t2;
  c = t0 - t2;
  if constexpr (!INV) {  // t1 - i t3, t1 + i t3
    b = mk(t1.x + t3.y, t1.y - t3.x);
    d = mk(t1.x - t3.y, t1.y + t3.x);
  } else {
    b = mk(t1.x - t3.y, t1.y + t3.x);
    d = mk(t1.x + t3.y, t1.y - t3.x);
  }
}

template <int R, bool INV>
__device__ __forceinline__ void dft(cf* v) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    cf a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
  } else if constexpr (R == 4) {
    radix4<INV>(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    cf e[4], o[4];
    sfor<4>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      e[k] = v[2 * k];
      o[k] = v[2 * k + 1];
    });
    dft<4, INV>(e);
    dft<4, INV>(o);
    sfor<4>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      cf t = twc<8, k, INV>(o[k]);
      v[k] = e[k] + t;
      v[k + 4] = e[k] - t;
    });
  } else {
    // radix-4 decimation in time: n = 4m + q
    constexpr int Q = R / 4;
    cf s0[Q], s1[Q], s2[Q], s3[Q];
    sfor<Q>([&](auto mc) {
      constexpr int m = decltype(mc)::value;
      s0[m] = v[4 * m + 0];
      s1[m] = v[4 * m + 1];
      s2[m] = v[4 * m + 2];
      s3[m] = v[4 * m + 3];
    });
    dft<Q, INV>(s0);
    dft<Q, INV>(s1);
    dft<Q, INV>(s2);
    dft<Q, INV>(s3);
    sfor<Q>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      cf a = s0[k];
      cf b = twc<R, k, INV>(s1[k]);
      cf c = twc<R, 2 * k, INV>(s2[k]);
      cf d = twc<R, 3 * k, INV>(s3[k]);
      radix4<INV>(a, b, c, d);
      v[k] = a;
      v[k + Q] = b;
      v[k + 2 * Q] = c;
      v[k + 3 * Q] = d;
    });
  }
}

// -------------------------------------------------------------------- plans
constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

// A plan: M = N/2 complex points, T threads, radices R0..R3 (0 = unused).
// R0 = P (one first-pass butterfly per thread), last radix = P/2 (two paired
// butterflies per thread), middle radices divide P.
template <int M_, int T_, int R0_, int R1_, int R2_, int R3_ = 0>
struct Plan {
  static constexpr int M = M_, T = T_, P = M_ / T_, N = 2 * M_;
  static constexpr int NP = R3_ ? 4 : 3;
  static constexpr int R[4] = {R0_, R1_, R2_, R3_};
  static constexpr int RL = NP == 4 ? R3_ : R2_;  // last radix
  static constexpr int PSH = ilog2c(R0_);          // LDS padding shift
  static constexpr int LDS = M + (M >> PSH);       // complex slots in LDS
  static_assert(R0_ == P, "first pass is one butterfly per thread");
  static_assert(2 * RL == P, "last pass is two butterflies per thread");
  static_assert(R0_ * R1_ * R2_ * (R3_ ? R3_ : 1) == M_, "radices multiply to M");
  static constexpr int ls(int p) { return p == 0 ? 1 : ls(p - 1) * R[p - 1]; }
  // Twiddle table (float2 entries), relative offsets:
  //  mid pass p (1..NP-2): W_{R_p Ls_p}^{r k} at [r * Ls_p + k], r < R_p, k < Ls_p
  //  last pass:            W_M^{r k} at [r * (T+1) + k], r < RL, k <= T
  //  post-processing:      W_N^{c + 2T q} at [q * (T+1) + c], q < RL, c <= T
  static constexpr int mid_off(int p) { return p <= 1 ? 0 : mid_off(p - 1) + R[p - 1] * ls(p - 1); }
  static constexpr int LAST_OFF = mid_off(NP - 1);
  static constexpr int POST_OFF = LAST_OFF + RL * (T + 1);
  static constexpr int TW_SIZE = POST_OFF + RL * (T + 1);
};

// The plan of each FFT size N = 2^L2, L2 = 9..15.  From N = 2048 on every
// plan holds 16 points per thread (T = N/32 threads), which leaves registers
// for prefetching the next operands while a transform runs.
constexpr int kMinL2 = 9, kMaxL2 = 15, kNumSizes = kMaxL2 - kMinL2 + 1;
template <int L2>
struct PlanFor;
template <>
struct PlanFor<9> {
  using type = Plan<256, 32, 8, 8, 4>;
};
template <>
struct PlanFor<10> {
  using type = Plan<512, 64, 8, 4, 4, 4>;
};
template <>
struct PlanFor<11> {
  using type = Plan<1024, 64, 16, 8, 8>;
};
template <>
struct PlanFor<12> {
  using type = Plan<2048, 128, 16, 16, 8>;
};
template <>
struct PlanFor<13> {
  using type = Plan<4096, 256, 16, 8, 4, 8>;
};
template <>
struct PlanFor<14> {
  using type = Plan<8192, 512, 16, 8, 8, 8>;
};
template <>
struct PlanFor<15> {
  using type = Plan<16384, 1024, 16, 16, 8, 8>;
};
template <int L2>
using PlanOf = typename PlanFor<L2>::type;

// Offset of each plan's table inside the one twiddle array.
template <int L2>
constexpr int tw_off() {
  if constexpr (L2 == kMinL2) return 0;
  else return tw_off<L2 - 1>() + PlanOf<L2 - 1>::TW_SIZE;
}
constexpr int kTwTotal = tw_off<kMaxL2 + 1>();

// Threads of the plan of size 2^l2 (0 outside 9..15).
__host__ __device__ constexpr int plan_threads(int l2) {
  return l2 == 9    ? PlanOf<9>::T
         : l2 == 10 ? PlanOf<10>::T
         : l2 == 11 ? PlanOf<11>::T
         : l2 == 12 ? PlanOf<12>::T
         : l2 == 13 ? PlanOf<13>::T
         : l2 == 14 ? PlanOf<14>::T
         : l2 == 15 ? PlanOf<15>::T
                    : 0;
}

// Calls f(PlanOf<L2>{}) for the runtime size l2 among the plans with T
// threads; with a single such plan the size is not tested.
template <int T, int L2 = kMinL2>
constexpr int plans_with_threads() {
  if constexpr (L2 > kMaxL2) return 0;
  else return (PlanOf<L2>::T == T ? 1 : 0) + plans_with_threads<T, L2 + 1>();
}
template <int T, int L2 = kMinL2, class F>
__device__ __forceinline__ void dispatch_plan(int l2, F&& f) {
  if constexpr (L2 <= kMaxL2) {
    if constexpr (PlanOf<L2>::T == T) {
      if (plans_with_threads<T>() == 1 || l2 == L2) {
        f(PlanOf<L2>{});
        return;
      }
    }
    dispatch_plan<T, L2 + 1>(l2, f);
  }
}

// LDS available to one workgroup's exchanges (the rest of the 160 KB of a
// CU is left for small shared arrays), and whether a plan of `lds` complex
// entries gets two exchange buffers.
constexpr int kLdsBudgetBytes = 160 * 1024 - 4096;
constexpr bool double_exchange(int lds) { return 2 * lds * 8 <= kLdsBudgetBytes; }

// Largest M and LDS footprint (exchange buffers) over the plans with T threads.
template <int T, int L2 = kMinL2>
constexpr int max_m_with_threads() {
  if constexpr (L2 > kMaxL2) return 0;
  else {
    constexpr int rest = max_m_with_threads<T, L2 + 1>();
    return PlanOf<L2>::T == T && PlanOf<L2>::M > rest ? PlanOf<L2>::M : rest;
  }
}
template <int T, int L2 = kMinL2>
constexpr int max_lds_with_threads() {
  if constexpr (L2 > kMaxL2) return 0;
  else {
    constexpr int rest = max_lds_with_threads<T, L2 + 1>();
    constexpr int mine = (double_exchange(PlanOf<L2>::LDS) ? 2 : 1) * PlanOf<L2>::LDS;
    return PlanOf<L2>::T == T && mine > rest ? mine : rest;
  }
}
// The same with one exchange buffer per plan.
template <int T, int L2 = kMinL2>
constexpr int max_lds_single_with_threads() {
  if constexpr (L2 > kMaxL2) return 0;
  else {
    constexpr int rest = max_lds_single_with_threads<T, L2 + 1>();
    return PlanOf<L2>::T == T && PlanOf<L2>::LDS > rest ? PlanOf<L2>::LDS : rest;
  }
}

template <class PL>
__device__ __forceinline__ int pad(int i) {
  return i + (i >> PL::PSH);
}

// ------------------------------------------------------------ the transforms
// Per-thread twiddle bases of a plan.  Every twiddle a thread applies is a
// power of one base per pass (the middle-pass butterflies of a thread share
// k = t mod Ls because T is a multiple of Ls), or, for the real
// post-processing, one base times a compile-time root of unity.  The bases are
// loaded once per utterance and the powers are formed in registers, so the
// transforms read no twiddle memory.
struct TwBase {
  cf mid[2];  // W_{R_p Ls_p}^{k}, k = t mod Ls_p, for middle passes p = 1, 2
  cf last;    // W_M^{kb}, kb = t (thread 0: T)
  cf post;    // W_N^{c}, c = t (thread 0: T)
};

// The LDS of a workgroup's data exchanges.  With room for two buffers
// (every plan but N = 32768) consecutive exchanges alternate between them:
// an exchange then needs one barrier (between its writes and its reads),
// because the buffer it writes was last read before the previous exchange's
// barrier.  With one buffer, a barrier also precedes the writes.  The parity
// is uniform across the workgroup and starts at 0 for each work item (the
// persistent loop's barriers separate items).  ONE asks for one buffer where
// two would fit, so that two workgroups share a CU's LDS.
template <class PL, bool ONE = false>
struct Xch {
  static constexpr bool kDouble = !ONE && double_exchange(PL::LDS);
  static constexpr int kEntries = (kDouble ? 2 : 1) * PL::LDS;
  cf* base;
  int par;
  __device__ cf* buf() const { return kDouble ? base + par * PL::LDS : base; }
  __device__ void before_write() const {
    if constexpr (!kDouble) __syncthreads();
  }
  __device__ void before_read() const { __syncthreads(); }
  __device__ void after_read() {
    if constexpr (kDouble) par ^= 1;
  }
};

// The exchange of a plan whose threads all belong to one wave (T <= 64), in
// a single buffer, synchronised at wave level only: the LDS executes one
// wave's operations in issue order, so a read issued after a write sees it
// and a write issued after a read does not disturb it; the fences only keep
// the compiler from moving the accesses across the exchange.  Several such
// groups can exchange independently inside a larger workgroup.
template <class PL>
struct XchWave {
  static_assert(PL::T <= 64, "one wave");
  static constexpr int kEntries = PL::LDS;
  cf* base;
  __device__ cf* buf() const { return base; }
  __device__ static void sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  __device__ void before_write() const { sync(); }
  __device__ void before_read() const { sync(); }
  __device__ void after_read() {}
};

template <class PL>
struct Fft {
  static constexpr int M = PL::M, T = PL::T, P = PL::P, NP = PL::NP, RL = PL::RL;
  static_assert(NP - 2 <= 2, "at most two middle passes");

  // LDS index strides after padding: every stride used below is a multiple
  // of 2^PSH, so pad(i + r s) = pad(i) + r ps(s).
  static constexpr int ps(int s) { return s + (s >> PL::PSH); }

  __device__ static __forceinline__ TwBase bases(const cf* __restrict__ tw_, int t) {
    const rsrc_t tw = make_rsrc(tw_, PL::TW_SIZE * 8);
    TwBase B;
    B.mid[0] = B.mid[1] = mk(1.f, 0.f);
    sfor<NP - 2>([&](auto pc) {
      constexpr int p = decltype(pc)::value + 1;
      constexpr int Ls = PL::ls(p);
      B.mid[p - 1] = ld2(tw, 8 * (t & (Ls - 1)), 8 * (PL::mid_off(p) + Ls));
    });
    const int kb = t ? t : T;
    B.last = ld2(tw, 8 * kb, 8 * (PL::LAST_OFF + (T + 1)));
    B.post = ld2(tw, 8 * kb, 8 * PL::POST_OFF);
    return B;
  }

  // Forward complex FFT.  In: v[r] = z[t + rT].  Out: slot layout (before the
  // real post-processing).  `lds` holds PL::LDS entries.  Contains barriers:
  // every thread of the workgroup must call it.
  template <class XC>
  __device__ static __forceinline__ void forward(cf* v, XC& X, const TwBase& B, int t_) {
    const int t = opaque_v(t_);
    // pass 0 (Ls = 1): no twiddles; outputs of butterfly t go to t*R0 + r
    dft<PL::R[0], false>(v);
    X.before_write();
    {
      cf* dst = X.buf() + t * (PL::R[0] + 1);
#pragma unroll
      for (int r = 0; r < PL::R[0]; ++r) dst[r] = v[r];
    }
    X.before_read();
    sfor<NP - 2>([&](auto pc) {
      constexpr int p = decltype(pc)::value + 1;
      constexpr int R = PL::R[p], Ls = PL::ls(p), NB = P / R;
      {
        const cf* lds = X.buf();
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const cf* src = lds + pad<PL>(t + T * b);
#pragma unroll
          for (int r = 0; r < R; ++r) v[b * R + r] = src[r * ps(M / R)];
        }
      }
      X.after_read();
      X.before_write();
      for_powers<R>(opaque_c(B.mid[p - 1]), [&](auto rc, cf w) {
        constexpr int r = decltype(rc)::value;
#pragma unroll
        for (int b = 0; b < NB; ++b) v[b * R + r] = cmul(v[b * R + r], w);
      });
      cf* lds = X.buf();
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = t + T * b;
        const int k = j & (Ls - 1);
        cf* u = v + b * R;
        dft<R, false>(u);
        cf* dst = lds + pad<PL>((j - k) * R + k);
#pragma unroll
        for (int r = 0; r < R; ++r) dst[r * ps(Ls)] = u[r];
      }
      X.before_read();
    });
    // last pass: butterflies ja, jb of radix RL, Ls = 2T.  Both use the
    // twiddles W_M^{r kb}: butterfly jb = 2T - t needs conj(W_M^{r t}) times
    // W_R^r, and the W_R^r factor is a rotation of its outputs by one bin.
    // Thread 0 (ja = 0, jb = T) uses W_M^{r T} for jb and 1 for ja.
    const int ja = t, jb = t ? 2 * T - t : T;
    const bool t0 = t == 0;
    cf a[RL], b[RL];
    {
      const cf* lds = X.buf();
      const cf* sa = lds + pad<PL>(ja);
      const cf* sb = lds + pad<PL>(jb);
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        a[r] = sa[r * ps(2 * T)];
        b[r] = sb[r * ps(2 * T)];
      }
    }
    X.after_read();
    for_powers<RL>(opaque_c(B.last), [&](auto rc, cf w) {
      constexpr int r = decltype(rc)::value;
      const cf aw = cmul(a[r], w);
      a[r] = t0 ? a[r] : aw;
      b[r] = cmulc(b[r], w);
    });
    dft<RL, false>(a);
    dft<RL, false>(b);
#pragma unroll
    for (int q = 0; q < RL; ++q) {
      v[q] = a[q];
      v[RL + q] = b[(q + 1) % RL];
    }
  }

  // Adjoint of forward(): slot layout in, v[r] = M * z[t + rT] out.
  template <class XC>
  __device__ static __forceinline__ void inverse(cf* v, XC& X, const TwBase& B, int t_) {
    const int t = opaque_v(t_);
    const int ja = t, jb = t ? 2 * T - t : T;
    const bool t0 = t == 0;
    cf a[RL], b[RL];
#pragma unroll
    for (int q = 0; q < RL; ++q) {
      a[q] = v[q];
      b[q] = v[RL + ((q + RL - 1) % RL)];
    }
    dft<RL, true>(a);
    dft<RL, true>(b);
    for_powers<RL>(opaque_c(B.last), [&](auto rc, cf w) {
      constexpr int r = decltype(rc)::value;
      const cf aw = cmulc(a[r], w);
      a[r] = t0 ? a[r] : aw;
      b[r] = cmul(b[r], w);
    });
    X.before_write();
    {
      cf* lds = X.buf();
      cf* da = lds + pad<PL>(ja);
      cf* db = lds + pad<PL>(jb);
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        da[r * ps(2 * T)] = a[r];
        db[r * ps(2 * T)] = b[r];
      }
    }
    X.before_read();
    sfor<NP - 2>([&](auto pc) {
      constexpr int p = NP - 2 - decltype(pc)::value;
      constexpr int R = PL::R[p], Ls = PL::ls(p), NB = P / R;
      {
        const cf* lds = X.buf();
#pragma unroll
        for (int bb = 0; bb < NB; ++bb) {
          const int j = t + T * bb;
          const int k = j & (Ls - 1);
          const cf* src = lds + pad<PL>((j - k) * R + k);
#pragma unroll
          for (int r = 0; r < R; ++r) v[bb * R + r] = src[r * ps(Ls)];
        }
      }
      X.after_read();
      X.before_write();
#pragma unroll
      for (int bb = 0; bb < NB; ++bb) dft<R, true>(v + bb * R);
      for_powers<R>(opaque_c(B.mid[p - 1]), [&](auto rc, cf w) {
        constexpr int r = decltype(rc)::value;
#pragma unroll
        for (int bb = 0; bb < NB; ++bb) v[bb * R + r] = cmulc(v[bb * R + r], w);
      });
      cf* lds = X.buf();
#pragma unroll
      for (int bb = 0; bb < NB; ++bb) {
        const int j = t + T * bb;
        cf* u = v + bb * R;
        cf* dst = lds + pad<PL>(j);
#pragma unroll
        for (int r = 0; r < R; ++r) dst[r * ps(M / R)] = u[r];
      }
      X.before_read();
    });
    {
      const cf* src = X.buf() + t * (PL::R[0] + 1);
#pragma unroll
      for (int r = 0; r < PL::R[0]; ++r) v[r] = src[r];
    }
    X.after_read();
    dft<PL::R[0], true>(v);
  }

  // Z[k], Z[M-k] and w = W_N^k -> 2 X[k], 2 X[M-k]:
  // E = Z[k] + conj(Z[M-k]), O = -i (Z[k] - conj(Z[M-k])), X = E + w O, X[M-k] = conj(E - w O)
  __device__ static __forceinline__ void post_pair(cf za, cf zb, cf w, cf& xa, cf& xb) {
    const cf E = mk(za.x + zb.x, za.y - zb.y);
    const cf O = mk(za.y + zb.y, zb.x - za.x);
    const cf wO = cmul(O, w);
    xa = E + wO;
    xb = mk(E.x - wO.x, wO.y - E.y);
  }
  // 2 Y[k], 2 Y[M-k] and w = W_N^k -> Z'[k], Z'[M-k] (twice the spectrum of
  // y[2n] + i y[2n+1]): E = Y[k] + conj(Y[M-k]), O = (Y[k] - conj(Y[M-k])) conj(w),
  // Z'[k] = E + i O, Z'[M-k] = conj(E) + i conj(O).
  __device__ static __forceinline__ void pre_pair(cf ya, cf yb, cf w, cf& za, cf& zb) {
    const cf E = mk(ya.x + yb.x, ya.y - yb.y);
    const cf D = mk(ya.x - yb.x, ya.y + yb.y);
    const cf O = cmulc(D, w);
    za = mk(E.x - O.y, E.y + O.x);
    zb = mk(E.x + O.y, O.x - E.y);
  }
  // Thread 0 owns the self-paired butterflies 0 and T: bins 2Tq pair with
  // 2T(R-q) (q = 0 is the DC / Nyquist pair, q = R/2 is bin M/2) and bins
  // T + 2Tq pair with T + 2T(R-1-q).  To keep every thread on the same code
  // path (a divergent branch would keep two copies of all data registers
  // live), thread 0's slots are permuted so that the generic pairing
  // (q, 2R-1-q) covers its pairs:
  //   slot q       <- b_q        (q < R/2)
  //   slot R + m   <- a_{m+1}    (m < R/2 - 1)
  //   slot 3R/2-1  <- a_0        (becomes the packed (X[0], X[N/2]) pair)
  // and slots R/2 (bin M/2) and 3R/2-1 are fixed up by selects.
  static constexpr int SP = 3 * RL / 2 - 1;  // thread 0's packed DC/Nyquist slot

  __device__ static __forceinline__ void perm_t0(cf* v, bool t0) {
    cf n0[RL / 2], n1[RL / 2];
#pragma unroll
    for (int q = 0; q < RL / 2; ++q) n0[q] = v[RL + q];
#pragma unroll
    for (int m = 0; m < RL / 2 - 1; ++m) n1[m] = v[m + 1];
    n1[RL / 2 - 1] = v[0];
#pragma unroll
    for (int q = 0; q < RL / 2; ++q) {
      v[q] = t0 ? n0[q] : v[q];
      v[RL + q] = t0 ? n1[q] : v[RL + q];
    }
  }
  __device__ static __forceinline__ void unperm_t0(cf* v, bool t0) {
    cf oa[RL / 2], ob[RL / 2];
#pragma unroll
    for (int q = 0; q < RL / 2; ++q) {
      oa[q] = q == 0 ? v[SP] : v[RL + q - 1];
      ob[q] = v[q];
    }
#pragma unroll
    for (int q = 0; q < RL / 2; ++q) {
      v[q] = t0 ? oa[q] : v[q];
      v[RL + q] = t0 ? ob[q] : v[RL + q];
    }
  }
  // Post-processing twiddles W_N^k of the first bin of each generic pair:
  // k = c + 2Tq with column c = t, except that thread 0 uses c = T for its
  // b-pairs (q < R/2) and c = 0 otherwise.  W_N^{c + 2Tq} = W_N^c W_{2R}^q.
  __device__ static __forceinline__ void post_twiddles(cf* w, const TwBase& B, bool t0) {
    const cf lo = opaque_c(B.post);
    const cf hi = t0 ? mk(1.f, 0.f) : lo;
    sfor<RL>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      w[q] = rot32<q * (32 / (2 * RL))>(q < RL / 2 ? lo : hi);
    });
  }

  // Real post-processing: Z (transform of x[2n] + i x[2n+1]) -> 2 X[k] in the
  // slot layout (thread 0 permuted as above).
  __device__ static __forceinline__ void post(cf* v, const TwBase& B, int t_) {
    const int t = opaque_v(t_);
    const bool t0 = t == 0;
    cf w[RL];
    post_twiddles(w, B, t0);
    const cf s0 = v[0], sh = v[RL / 2];
    perm_t0(v, t0);
#pragma unroll
    for (int q = 0; q < RL; ++q) {
      cf xa, xb;
      post_pair(v[q], v[2 * RL - 1 - q], w[q], xa, xb);
      v[q] = xa;
      v[2 * RL - 1 - q] = xb;
    }
    // thread 0: (2 X[0], 2 X[N/2]) = 2 (Re + Im, Re - Im) of Z[0]; 2 X[M/2] = 2 conj(Z[M/2])
    const cf dc = mk(2.f * (s0.x + s0.y), 2.f * (s0.x - s0.y));
    const cf mid = mk(2.f * sh.x, -2.f * sh.y);
    v[SP] = t0 ? dc : v[SP];
    v[RL / 2] = t0 ? mid : v[RL / 2];
  }

  // Inverse of post() up to a factor 2: 2 Y[k] (slot layout) -> Z' such that
  // inverse() returns 4 M y.
  __device__ static __forceinline__ void pre(cf* v, const TwBase& B, int t_) {
    const int t = opaque_v(t_);
    const bool t0 = t == 0;
    cf w[RL];
    post_twiddles(w, B, t0);
    const cf d = v[SP], sh = v[RL / 2];
#pragma unroll
    for (int q = 0; q < RL; ++q) {
      cf za, zb;
      pre_pair(v[q], v[2 * RL - 1 - q], w[q], za, zb);
      v[q] = za;
      v[2 * RL - 1 - q] = zb;
    }
    // thread 0: Z'[0] = (Y0 + YN/2) + i (Y0 - YN/2); Z'[M/2] = 2 conj(Y[M/2])
    const cf z0 = mk(d.x + d.y, d.x - d.y);
    const cf zm = mk(2.f * sh.x, -2.f * sh.y);
    v[SP] = t0 ? z0 : v[SP];
    v[RL / 2] = t0 ? zm : v[RL / 2];
    unperm_t0(v, t0);
  }
};

// Host-side twiddle generation (FP64, rounded once to float).  Fills `out`
// (kTwTotal float2) with every plan's table.
void fill_twiddles(float* out);

}  // namespace rsim

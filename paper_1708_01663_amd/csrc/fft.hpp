// Stockham complex FFT held in registers, exchanged through LDS between
// radix passes (gfx950).
//
// One transform of length P is processed by NT cooperating threads; each
// thread owns V = P/NT points.  A pass of radix R (stride Ns = product of the
// radices already applied) consists of P/R butterflies; butterfly j reads
// in[j + r*P/R], multiplies by the twiddles w^(r*k), k = j mod Ns,
// w = exp(-+2 pi i/(Ns R)), applies the radix-R DFT, and writes
// out[(j/Ns)*Ns*R + k + r*Ns].  The result of the last pass lands in natural
// order.  Thread t owns butterflies j = t + b*NT of every pass, so its
// registers hold in[j + r*P/R] before the first pass and out[j + r*P/R_last]
// after the last one; the kernels load and store straight from and to global
// memory in those layouts, and LDS is touched only between passes.
//
// A forward transform followed by an inverse whose first radix equals the
// forward's last radix needs no exchange in between: the values a thread
// holds after the forward are exactly the inputs it needs.
#pragma once

#include "common.hpp"

namespace cisor {

template <int... Rs> struct RadixList {};

// ---- radix-R DFTs; DIR = -1 forward (exp(-i...)), +1 inverse ----

template <int DIR, typename C> __device__ __forceinline__ void dft2(C &a, C &b) {
  C t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int DIR, typename C> __device__ __forceinline__ void dft4(C &v0, C &v1, C &v2, C &v3) {
  C a = cadd(v0, v2), b = csub(v0, v2);
  C c = cadd(v1, v3), d = cmul_si(csub(v1, v3), DIR);  // DIR*i*(v1 - v3)
  v0 = cadd(a, c);
  v2 = csub(a, c);
  v1 = cadd(b, d);
  v3 = csub(b, d);
}

template <int DIR, typename C> __device__ __forceinline__ void dft8(C *v) {
  using R = real_t<C>;
  // even / odd halves
  C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  const R s = static_cast<R>(0.70710678118654752440084436210485);
  // w8^1 = (1 + DIR i)/sqrt2, w8^2 = DIR i, w8^3 = (-1 + DIR i)/sqrt2
  C t1 = cscale(cadd(o1, cmul_si(o1, DIR)), s);
  C t2 = cmul_si(o2, DIR);
  C t3 = cscale(csub(cmul_si(o3, DIR), o3), s);
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, t1);
  v[5] = csub(e1, t1);
  v[2] = cadd(e2, t2);
  v[6] = csub(e2, t2);
  v[3] = cadd(e3, t3);
  v[7] = csub(e3, t3);
}

template <int DIR, typename C> __device__ __forceinline__ void dft3(C &v0, C &v1, C &v2) {
  using R = real_t<C>;
  const R h = static_cast<R>(0.86602540378443864676372317075294);  // sqrt(3)/2
  C t1 = cadd(v1, v2);
  C t2 = cscale(cmul_si(csub(v1, v2), DIR), h);  // DIR*i*sqrt3/2*(v1 - v2)
  C m = csub(v0, cscale(t1, static_cast<R>(0.5)));
  v0 = cadd(v0, t1);
  v1 = cadd(m, t2);
  v2 = csub(m, t2);
}

// Pruned radix-R DFTs of the first and last passes.  In a zero-padded
// transform (input zero from P/2 on) the first pass's inputs r >= R/2 are zero
// (HALF_IN); in a cropped one (outputs kept below P/2 only) the last pass's
// outputs r >= R/2 are never used (HALF_OUT, left unspecified).  R even.
enum : int { PRUNE_NONE = 0, PRUNE_IN = 1, PRUNE_OUT = 2 };

template <int DIR, typename C> __device__ __forceinline__ void dft4_half_in(C &v0, C &v1, C &v2, C &v3) {
  // inputs (v0, v1, 0, 0)
  const C a = v0, c = v1, d = cmul_si(v1, DIR);
  v0 = cadd(a, c);
  v2 = csub(a, c);
  v1 = cadd(a, d);
  v3 = csub(a, d);
}

template <int R, int DIR, int PRUNE, typename C> __device__ __forceinline__ void dft_pruned(C *v) {
  if constexpr (PRUNE == PRUNE_IN) {
    if constexpr (R == 2) {
      v[1] = v[0];
    } else if constexpr (R == 4) {
      dft4_half_in<DIR>(v[0], v[1], v[2], v[3]);
    } else {
      static_assert(R == 8, "pruned radix must be 2, 4 or 8");
      using Rr = real_t<C>;
      C e0 = v[0], e1 = v[2], e2, e3, o0 = v[1], o1 = v[3], o2, o3;
      dft4_half_in<DIR>(e0, e1, e2, e3);
      dft4_half_in<DIR>(o0, o1, o2, o3);
      const Rr s = static_cast<Rr>(0.70710678118654752440084436210485);
      const C t1 = cscale(cadd(o1, cmul_si(o1, DIR)), s);
      const C t2 = cmul_si(o2, DIR);
      const C t3 = cscale(csub(cmul_si(o3, DIR), o3), s);
      v[0] = cadd(e0, o0);
      v[4] = csub(e0, o0);
      v[1] = cadd(e1, t1);
      v[5] = csub(e1, t1);
      v[2] = cadd(e2, t2);
      v[6] = csub(e2, t2);
      v[3] = cadd(e3, t3);
      v[7] = csub(e3, t3);
    }
  } else {
    if constexpr (R == 2) {
      v[0] = cadd(v[0], v[1]);
    } else if constexpr (R == 4) {
      const C a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
      const C c = cadd(v[1], v[3]), d = cmul_si(csub(v[1], v[3]), DIR);
      v[0] = cadd(a, c);
      v[1] = cadd(b, d);
    } else {
      static_assert(R == 8, "pruned radix must be 2, 4 or 8");
      using Rr = real_t<C>;
      C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
      C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
      dft4<DIR>(e0, e1, e2, e3);
      dft4<DIR>(o0, o1, o2, o3);
      const Rr s = static_cast<Rr>(0.70710678118654752440084436210485);
      v[0] = cadd(e0, o0);
      v[1] = cadd(e1, cscale(cadd(o1, cmul_si(o1, DIR)), s));
      v[2] = cadd(e2, cmul_si(o2, DIR));
      v[3] = cadd(e3, cscale(csub(cmul_si(o3, DIR), o3), s));
    }
  }
}

template <int R, int DIR, typename C> __device__ __forceinline__ void dft(C *v) {
  if constexpr (R == 2) {
    dft2<DIR>(v[0], v[1]);
  } else if constexpr (R == 3) {
    dft3<DIR>(v[0], v[1], v[2]);
  } else if constexpr (R == 4) {
    dft4<DIR>(v[0], v[1], v[2], v[3]);
  } else {
    static_assert(R == 8, "radix must be 2, 3, 4 or 8");
    dft8<DIR>(v);
  }
}

// Twiddles.  Butterfly j of a pass with stride Ns needs w^(r k), r = 1..R-1,
// k = j mod Ns, w = exp(-+2 pi i/(Ns R)).  Only w^k, w^2k and w^4k are read
// from the table (tw[m] = exp(-2 pi i m / P), conjugated for the inverse);
// the other powers are products of at most two of them, so each is within a
// few ulp of the tabulated value while the table traffic drops from R-1
// gathers to at most 3.  When NT is a multiple of Ns every butterfly of a
// thread has the same k and one set serves them all.
//
// Two sources implement fetch(b, w1, w2, w4) for butterfly b of a pass:
//  * Tw: every pass's values loaded into registers at once (issued at kernel
//    entry, so their latency overlaps with the data loads);
//  * TwLazy: read from a table (e.g. an LDS copy) when the pass runs, which
//    costs no registers across passes.
template <typename C, int DIR> __device__ __forceinline__ C tw_read(const C *__restrict__ tab, int m) {
  C x = tab[m];
  if constexpr (DIR > 0) x.y = -x.y;
  return x;
}

template <typename C, int P, int NT, int DIR, int Ns, typename List> struct Tw;
template <typename C, int P, int NT, int DIR, int Ns> struct Tw<C, P, NT, DIR, Ns, RadixList<>> {
  __device__ __forceinline__ void load(int, const C *__restrict__) {}
};
template <typename C, int P, int NT, int DIR, int Ns, int R, int... Rest>
struct Tw<C, P, NT, DIR, Ns, RadixList<R, Rest...>> {
  static constexpr int BPT = P / (R * NT);
  static constexpr bool SHARED_K = (NT % Ns) == 0;
  static constexpr int NW = (Ns == 1) ? 0 : (SHARED_K ? 1 : BPT);
  static constexpr int STEP = P / (Ns * R);
  C w[NW > 0 ? NW : 1][3];
  Tw<C, P, NT, DIR, Ns * R, RadixList<Rest...>> next;
  __device__ __forceinline__ void load(int tid, const C *__restrict__ tab) {
    if constexpr (NW > 0) {
#pragma unroll
      for (int b = 0; b < NW; ++b) {
        const int k = (SHARED_K ? tid : tid + b * NT) % Ns;
        w[b][0] = tw_read<C, DIR>(tab, k * STEP);
        if constexpr (R >= 3) w[b][1] = tw_read<C, DIR>(tab, 2 * k * STEP);
        if constexpr (R == 8) w[b][2] = tw_read<C, DIR>(tab, 4 * k * STEP);
      }
    }
    next.load(tid, tab);
  }
  __device__ __forceinline__ void fetch(int b, C &w1, C &w2, C &w4) const {
    const int wb = SHARED_K ? 0 : b;
    w1 = w[wb][0];
    if constexpr (R >= 3) w2 = w[wb][1];
    if constexpr (R == 8) w4 = w[wb][2];
  }
  __device__ __forceinline__ const Tw<C, P, NT, DIR, Ns * R, RadixList<Rest...>> &next_node() const { return next; }
};

template <typename C, int P, int NT, int DIR, int Ns, typename List> struct TwLazy;
template <typename C, int P, int NT, int DIR, int Ns> struct TwLazy<C, P, NT, DIR, Ns, RadixList<>> {
  const C *tab;
  int tid;
};
template <typename C, int P, int NT, int DIR, int Ns, int R, int... Rest>
struct TwLazy<C, P, NT, DIR, Ns, RadixList<R, Rest...>> {
  static constexpr bool SHARED_K = (NT % Ns) == 0;
  static constexpr int STEP = P / (Ns * R);
  const C *tab;
  int tid;
  __device__ __forceinline__ void fetch(int b, C &w1, C &w2, C &w4) const {
    const int k = (SHARED_K ? tid : tid + b * NT) % Ns;
    w1 = tw_read<C, DIR>(tab, k * STEP);
    if constexpr (R >= 3) w2 = tw_read<C, DIR>(tab, 2 * k * STEP);
    if constexpr (R == 8) w4 = tw_read<C, DIR>(tab, 4 * k * STEP);
  }
  __device__ __forceinline__ TwLazy<C, P, NT, DIR, Ns * R, RadixList<Rest...>> next_node() const { return {tab, tid}; }
};

//  * TwPass: per-pass tables in LDS holding every power a butterfly needs,
//    laid out [r][k] (slot r of the pass's Ns values of k holds w^(r k)), so
//    that one address serves the R - 1 reads (LDS reads with immediate
//    offsets r Ns) and no product is formed; lanes with consecutive k read
//    consecutive entries, so a wave whose lanes hold different k reads without
//    bank conflicts.  The tables hold the forward
//    (exp(-2 pi i ...)) values; the inverse multiplies by their conjugates.
//    TwPassLayout gives each pass's offset; tw_pass_build fills the tables
//    from the length-P table.
template <int Ns, typename List> struct TwPassLayout;
template <int Ns> struct TwPassLayout<Ns, RadixList<>> {
  static constexpr int SIZE = 0;
};
template <int Ns, int R, int... Rest> struct TwPassLayout<Ns, RadixList<R, Rest...>> {
  static constexpr int HERE = Ns > 1 ? Ns * 8 : 0;   // complex entries of this pass's table
  using Next = TwPassLayout<Ns * R, RadixList<Rest...>>;
  static constexpr int SIZE = HERE + Next::SIZE;
};

template <typename C, int P, int Ns, typename List> struct TwPassBuild {
  __device__ static __forceinline__ void run(C *, const C *__restrict__, int, int) {}
};
template <typename C, int P, int Ns, int R, int... Rest> struct TwPassBuild<C, P, Ns, RadixList<R, Rest...>> {
  __device__ static __forceinline__ void run(C *tab, const C *__restrict__ tw, int t0, int nt) {
    if constexpr (Ns > 1) {
      constexpr int STEP = P / (Ns * R);
      for (int i = t0; i < Ns * 8; i += nt) {
        const int r = i / Ns, k = i % Ns;
        if (r < R) tab[i] = tw[r * k * STEP];   // r k STEP < P
      }
    }
    TwPassBuild<C, P, Ns * R, RadixList<Rest...>>::run(tab + TwPassLayout<Ns, RadixList<R, Rest...>>::HERE, tw, t0,
                                                        nt);
  }
};
// Fill the pass tables of a radix list from tw[m] = exp(-2 pi i m / P)
// (threads t0, t0 + nt, ...).
template <typename C, int P, typename List>
__device__ __forceinline__ void tw_pass_build(C *tab, const C *__restrict__ tw, int t0, int nt) {
  TwPassBuild<C, P, 1, List>::run(tab, tw, t0, nt);
}

template <typename C, int P, int NT, int DIR, int Ns, typename List> struct TwPass;
template <typename C, int P, int NT, int DIR, int Ns> struct TwPass<C, P, NT, DIR, Ns, RadixList<>> {
  const C *tab;
  int tid;
};
template <typename C, int P, int NT, int DIR, int Ns, int R, int... Rest>
struct TwPass<C, P, NT, DIR, Ns, RadixList<R, Rest...>> {
  static constexpr bool FULL = true;
  static constexpr bool SHARED_K = (NT % Ns) == 0;
  const C *tab;   // this pass's table
  int tid;
  __device__ __forceinline__ void fetch_all(int b, C (&w)[8]) const {
    const int k = (SHARED_K ? tid : tid + b * NT) % Ns;
    const C *p = tab + k;
#pragma unroll
    for (int r = 1; r < R; ++r) w[r] = p[r * Ns];
  }
  __device__ __forceinline__ TwPass<C, P, NT, DIR, Ns * R, RadixList<Rest...>> next_node() const {
    return {tab + TwPassLayout<Ns, RadixList<R, Rest...>>::HERE, tid};
  }
};

template <typename TW, typename = void> struct tw_is_full { static constexpr bool value = false; };
template <typename TW> struct tw_is_full<TW, decltype((void)TW::FULL, void())> {
  static constexpr bool value = TW::FULL;
};

// Twiddle + DFT for every butterfly a thread owns in one pass (PRUNE: see
// dft_pruned; only for even radices).
template <typename C, int P, int NT, int R, int Ns, int DIR, typename TW, int PRUNE = PRUNE_NONE>
__device__ __forceinline__ void pass_compute(C (&v)[P / NT], const TW &t) {
  constexpr int BPT = P / (R * NT);
  constexpr bool SHARED_K = (NT % Ns) == 0;
  C w[8];
  if constexpr (tw_is_full<TW>::value) {
    // every power read from the pass table; the inverse multiplies by the
    // conjugate of the forward value (same instruction count as a product)
    if constexpr (Ns > 1 && SHARED_K) t.fetch_all(0, w);
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      if constexpr (Ns > 1) {
        if constexpr (!SHARED_K) t.fetch_all(b, w);
#pragma unroll
        for (int r = 1; r < R; ++r) v[b * R + r] = DIR < 0 ? cmul(v[b * R + r], w[r]) : cmulc(w[r], v[b * R + r]);
      }
      if constexpr (PRUNE != PRUNE_NONE && R % 2 == 0)
        dft_pruned<R, DIR, PRUNE>(&v[b * R]);
      else
        dft<R, DIR>(&v[b * R]);
    }
  } else {
    auto make = [&](int b) {
      C w1 = {}, w2 = {}, w4 = {};
      t.fetch(b, w1, w2, w4);
      w[1] = w1;
      if constexpr (R >= 3) w[2] = w2;
      if constexpr (R == 4) w[3] = cmul(w[1], w[2]);
      if constexpr (R == 8) {
        w[4] = w4;
        w[3] = cmul(w[1], w[2]);
        w[5] = cmul(w[1], w[4]);
        w[6] = cmul(w[2], w[4]);
        w[7] = cmul(w[3], w[4]);
      }
    };
    if constexpr (Ns > 1 && SHARED_K) make(0);
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      if constexpr (Ns > 1) {
        if constexpr (!SHARED_K) make(b);
#pragma unroll
        for (int r = 1; r < R; ++r) v[b * R + r] = cmul(v[b * R + r], w[r]);
      }
      if constexpr (PRUNE != PRUNE_NONE && R % 2 == 0)
        dft_pruned<R, DIR, PRUNE>(&v[b * R]);
      else
        dft<R, DIR>(&v[b * R]);
    }
  }
}

// Synchronisation between the LDS exchanges of a transform: the whole block
// (threads of one transform spread over several waves), or one wave (every
// thread of the transform in the same wave; LDS operations of a wave complete
// in order, so only the compiler must be kept from reordering them).
struct BlockSync {
  __device__ static __forceinline__ void sync() { __syncthreads(); }
};
struct WaveSync {
  __device__ static __forceinline__ void sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
};

// LDS index of transform element i.  PAD 1: one complex of padding after
// every 32 (a transform held contiguously, stride ls = 1, would otherwise
// send the stride-Ns writes of a pass to a few banks); a transform of length
// P then occupies lds_span(P) elements.  PAD 2: one element of padding after
// every 16 (P + P/16 elements; power-of-two P): with ls = 8 interleaved
// columns, the first pass's writes of rows 8 tid + r by the eight row offsets
// of a wave would otherwise share 16 banks.
template <int PAD> __device__ __forceinline__ int lds_index(int i) {
  return PAD == 1 ? i + (i >> 5) : (PAD == 2 ? i + (i >> 4) : i);
}
__host__ __device__ constexpr int lds_span(int P) { return P + P / 32; }
// With PAD 2, lds_index(i + d) = lds_index(i) + pad_step<2>(d) whenever
// [i, i + d] crosses no more multiples of 16 than [0, d] (PAD 1: of 32).  That
// holds for both sides of every exchange of a power-of-two transform: a
// butterfly's writes start at an offset k < Ns inside a group aligned to Ns R
// (d = r Ns), and a pass's reads start at j < P / R2 (d = r P / R2).  So for
// power-of-two lengths a thread forms one padded index per butterfly and the
// rest are compile-time offsets.
template <int PAD> __host__ __device__ constexpr int pad_step(int d) {
  return PAD == 1 ? d + d / 32 : (PAD == 2 ? d + d / 16 : d);
}

// PI: the input is zero from P/2 on (prune the first pass); PO: only outputs
// below P/2 are used (prune the last pass).  The twiddle multiply of the last
// pass still covers every input (they all feed the kept outputs).
template <typename C, int P, int NT, int DIR, int Ns, typename List, typename SY = BlockSync, int PAD = 0,
          bool PI = false, bool PO = false>
struct Stockham;

template <typename C, int P, int NT, int DIR, int Ns, int R, typename SY, int PAD, bool PI, bool PO>
struct Stockham<C, P, NT, DIR, Ns, RadixList<R>, SY, PAD, PI, PO> {
  static constexpr int LAST = R;
  template <typename TW>
  __device__ static __forceinline__ void run(C (&v)[P / NT], int tid, C *lds, int ls, const TW &t) {
    static_assert(Ns * R == P, "radices must multiply to P");
    static_assert(!PI, "a single-pass plan cannot be pruned at both ends");
    pass_compute<C, P, NT, R, Ns, DIR, TW, PO ? PRUNE_OUT : PRUNE_NONE>(v, t);
  }
};

template <typename C, int P, int NT, int DIR, int Ns, int R, int R2, int... Rest, typename SY, int PAD, bool PI,
          bool PO>
struct Stockham<C, P, NT, DIR, Ns, RadixList<R, R2, Rest...>, SY, PAD, PI, PO> {
  using Next = Stockham<C, P, NT, DIR, Ns * R, RadixList<R2, Rest...>, SY, PAD, false, PO>;
  static constexpr int LAST = Next::LAST;
  template <typename TW>
  __device__ static __forceinline__ void run(C (&v)[P / NT], int tid, C *lds, int ls, const TW &t) {
    static_assert(P % (R * NT) == 0 && P % (R2 * NT) == 0, "NT must divide every pass");
    pass_compute<C, P, NT, R, Ns, DIR, TW, PI ? PRUNE_IN : PRUNE_NONE>(v, t);
    constexpr int BPT = P / (R * NT);
#pragma unroll
    for (int b = 0; b < BPT; ++b) {
      const int j = tid + b * NT;
      const int k = j % Ns;
      const int base = (j / Ns) * Ns * R + k;
      static_assert(PAD != 2 || (P & (P - 1)) == 0, "PAD 2 needs a power-of-two length");
      if constexpr (PAD != 0 && (P & (P - 1)) == 0) {
        C *const pb = lds + lds_index<PAD>(base) * ls;
#pragma unroll
        for (int r = 0; r < R; ++r) pb[pad_step<PAD>(r * Ns) * ls] = v[b * R + r];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) lds[lds_index<PAD>(base + r * Ns) * ls] = v[b * R + r];
      }
    }
    SY::sync();
    constexpr int BPT2 = P / (R2 * NT);
#pragma unroll
    for (int b = 0; b < BPT2; ++b) {
      const int j = tid + b * NT;
      if constexpr (PAD != 0 && (P & (P - 1)) == 0) {
        const C *const pb = lds + lds_index<PAD>(j) * ls;
#pragma unroll
        for (int r = 0; r < R2; ++r) v[b * R2 + r] = pb[pad_step<PAD>(r * (P / R2)) * ls];
      } else {
#pragma unroll
        for (int r = 0; r < R2; ++r) v[b * R2 + r] = lds[lds_index<PAD>(j + r * (P / R2)) * ls];
      }
    }
    SY::sync();
    Next::run(v, tid, lds, ls, t.next_node());
  }
};

template <typename List> struct FirstRadix;
template <int R, int... Rest> struct FirstRadix<RadixList<R, Rest...>> { static constexpr int value = R; };

// Per-length plan.  fwd/inv are mirror images so that a forward transform
// can feed an inverse one in registers.  NT_ROW threads per row transform
// (8 points per thread for powers of two, 24 for lengths with a factor 3).
template <int P> struct Plan;
template <> struct Plan<64> {
  using fwd = RadixList<8, 8>;
  using inv = RadixList<8, 8>;
  static constexpr int NT_ROW = 8;
};
template <> struct Plan<128> {
  using fwd = RadixList<2, 8, 8>;
  using inv = RadixList<8, 8, 2>;
  static constexpr int NT_ROW = 16;
};
template <> struct Plan<192> {
  using fwd = RadixList<3, 8, 8>;
  using inv = RadixList<8, 8, 3>;
  static constexpr int NT_ROW = 8;
};
template <> struct Plan<256> {
  using fwd = RadixList<4, 8, 8>;
  using inv = RadixList<8, 8, 4>;
  static constexpr int NT_ROW = 32;
};
template <> struct Plan<384> {
  using fwd = RadixList<3, 2, 8, 8>;
  using inv = RadixList<8, 8, 2, 3>;
  static constexpr int NT_ROW = 16;
};
template <> struct Plan<512> {
  using fwd = RadixList<8, 8, 8>;
  using inv = RadixList<8, 8, 8>;
  static constexpr int NT_ROW = 64;
};
template <> struct Plan<768> {
  using fwd = RadixList<3, 4, 8, 8>;
  using inv = RadixList<8, 8, 4, 3>;
  static constexpr int NT_ROW = 32;
};
template <> struct Plan<1024> {
  using fwd = RadixList<2, 8, 8, 8>;
  using inv = RadixList<8, 8, 8, 2>;
  static constexpr int NT_ROW = 128;
};

// Alternative radix plans (same lengths, other factorisations), used by the
// column-kernel variants that the autotuner picks from.
template <int P> struct PlanAlt;
template <> struct PlanAlt<64> {
  using fwd = RadixList<4, 4, 4>;
  using inv = RadixList<4, 4, 4>;
};
template <> struct PlanAlt<128> {
  using fwd = RadixList<4, 4, 8>;
  using inv = RadixList<8, 4, 4>;
};
template <> struct PlanAlt<192> {
  using fwd = RadixList<3, 4, 4, 4>;
  using inv = RadixList<4, 4, 4, 3>;
};
template <> struct PlanAlt<256> {
  using fwd = RadixList<4, 4, 4, 4>;
  using inv = RadixList<4, 4, 4, 4>;
};
template <> struct PlanAlt<384> {
  using fwd = RadixList<3, 4, 4, 8>;
  using inv = RadixList<8, 4, 4, 3>;
};
template <> struct PlanAlt<512> {
  using fwd = RadixList<2, 4, 8, 8>;
  using inv = RadixList<8, 8, 4, 2>;
};
template <> struct PlanAlt<768> {
  using fwd = RadixList<3, 4, 4, 4, 4>;
  using inv = RadixList<4, 4, 4, 4, 3>;
};
template <> struct PlanAlt<1024> {
  using fwd = RadixList<4, 4, 8, 8>;
  using inv = RadixList<8, 8, 4, 4>;
};
template <int P, int PV> struct PlanSel { using type = Plan<P>; };
template <int P> struct PlanSel<P, 1> { using type = PlanAlt<P>; };

// Twiddle sources of a whole transform (all passes) of length P by NT threads.
template <typename C, int P, int NT, int DIR, typename List> using TwSet = Tw<C, P, NT, DIR, 1, List>;
template <typename C, int P, int NT, int DIR, typename List> using TwTable = TwLazy<C, P, NT, DIR, 1, List>;

template <typename C, int P, int NT, int DIR, typename List, typename TW, typename SY = BlockSync, int PAD = 0,
          bool PI = false, bool PO = false>
__device__ __forceinline__ void fft_regs(C (&v)[P / NT], int tid, C *lds, int ls, const TW &t) {
  Stockham<C, P, NT, DIR, 1, List, SY, PAD, PI, PO>::run(v, tid, lds, ls, t);
}

}  // namespace cisor

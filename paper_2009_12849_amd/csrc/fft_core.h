// Device FFT building blocks for gfx950: complex helpers, radix-2/3/4/8
// butterflies, and two Stockham engines sharing them:
//   * CtFft<T, N, NT, INV>: length fixed at compile time, NT threads per
//     transform, every index folded to constants; values stay in registers
//     inside a pass and cross threads through LDS between passes. The first
//     pass takes its inputs from the caller's registers and the last pass
//     leaves its outputs there, so the kernels read global memory straight
//     into the first pass and write the last pass straight to global memory.
//   * fft_lds(): runtime length (any 2^a 3^b), whole transform in LDS; the
//     fallback for lengths without a compile-time instance.
// Twiddles exp(-2 pi i t/N) come from a per-plan table built on the host.
#pragma once
#include <hip/hip_runtime.h>

#include "monc_types.h"

namespace monc {

template <typename T> struct V2;
template <> struct V2<float> { using t = float2; };
template <> struct V2<double> { using t = double2; };
template <typename T> using cx = typename V2<T>::t;

// Twiddle table read through a global-address-space pointer: the table
// pointer sits in a member descriptor, where it is a generic pointer that
// would otherwise become a flat load (which also holds up LDS waits).
template <typename C> __device__ __forceinline__ C load_tw(const C* p) {
  using E = decltype(C{}.x);
  typedef E pair __attribute__((ext_vector_type(2)));
  const pair v = *(const __attribute__((address_space(1))) pair*)p;
  return C{v.x, v.y};
}

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C> __device__ __forceinline__ C cmulconj(C a, C b) {  // a * conj(b)
  return C{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename C> __device__ __forceinline__ C mul_mi(C a) { return C{a.y, -a.x}; }  // -i a
template <typename C> __device__ __forceinline__ C mul_pi(C a) { return C{-a.y, a.x}; }  // +i a

// ---------------------------------------------------------------------------
// small DFTs (forward: exp(-2 pi i rs/R); inverse: exp(+2 pi i rs/R))
// ---------------------------------------------------------------------------
template <bool INV, typename C> __device__ __forceinline__ void dft2(C* v) {
  C a = v[0];
  v[0] = cadd(a, v[1]);
  v[1] = csub(a, v[1]);
}

template <bool INV, typename C> __device__ __forceinline__ void dft4(C& x0, C& x1, C& x2, C& x3) {
  C a = cadd(x0, x2), b = csub(x0, x2), c = cadd(x1, x3), d = csub(x1, x3);
  C jd = INV ? mul_pi(d) : mul_mi(d);
  x0 = cadd(a, c);
  x2 = csub(a, c);
  x1 = cadd(b, jd);
  x3 = csub(b, jd);
}

template <bool INV, typename C> __device__ __forceinline__ void dft8(C* v) {
  using T = decltype(v[0].x);
  const T h = (T)0.70710678118654752440;  // sqrt(1/2)
  C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<INV>(e0, e1, e2, e3);
  dft4<INV>(o0, o1, o2, o3);
  C t1, t2, t3;  // o_s * W8^(+-s)
  if (!INV) {
    t1 = C{h * (o1.x + o1.y), h * (o1.y - o1.x)};
    t2 = mul_mi(o2);
    t3 = C{h * (o3.y - o3.x), -h * (o3.x + o3.y)};
  } else {
    t1 = C{h * (o1.x - o1.y), h * (o1.x + o1.y)};
    t2 = mul_pi(o2);
    t3 = C{-h * (o3.x + o3.y), h * (o3.x - o3.y)};
  }
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, t1);
  v[5] = csub(e1, t1);
  v[2] = cadd(e2, t2);
  v[6] = csub(e2, t2);
  v[3] = cadd(e3, t3);
  v[7] = csub(e3, t3);
}

template <bool INV, typename C> __device__ __forceinline__ void dft3(C* v) {
  using T = decltype(v[0].x);
  const T s3 = (T)0.86602540378443864676;  // sin(2 pi/3)
  C s = cadd(v[1], v[2]);
  C d = csub(v[1], v[2]);
  C t = C{v[0].x - (T)0.5 * s.x, v[0].y - (T)0.5 * s.y};
  C sd = C{s3 * d.x, s3 * d.y};
  C jsd = INV ? mul_pi(sd) : mul_mi(sd);
  v[0] = cadd(v[0], s);
  v[1] = cadd(t, jsd);
  v[2] = csub(t, jsd);
}

// a * W16^E (forward: exp(-2 pi i E/16); inverse: its conjugate), E = 0..15
template <int E, bool INV, typename C> __device__ __forceinline__ C w16(C a) {
  using T = decltype(a.x);
  constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173;  // cos, sin(pi/8)
  constexpr double h = 0.70710678118654752440;
  constexpr double cs[16] = {1, c1, h, s1, 0, -s1, -h, -c1, -1, -c1, -h, -s1, 0, s1, h, c1};
  constexpr double sn[16] = {0, s1, h, c1, 1, c1, h, s1, 0, -s1, -h, -c1, -1, -c1, -h, -s1};
  if constexpr (E == 0) return a;
  else if constexpr (E == 4) return INV ? mul_pi(a) : mul_mi(a);
  else if constexpr (E == 8) return C{-a.x, -a.y};
  else {
    const T c = (T)cs[E], sv = INV ? (T)sn[E] : -(T)sn[E];  // multiply by c + i sv
    return C{a.x * c - a.y * sv, a.x * sv + a.y * c};
  }
}

// 16-point DFT as 4 x 4: DFT4 over n1 of x[4 n1 + n2], twiddle W16^(n2 k1),
// DFT4 over n2; output k1 + 4 k2 in natural order.
template <bool INV, typename C> __device__ __forceinline__ void dft16(C* v) {
  C y[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    C a = v[n2], b = v[4 + n2], c = v[8 + n2], d = v[12 + n2];
    dft4<INV>(a, b, c, d);
    y[n2][0] = a;
    y[n2][1] = b;
    y[n2][2] = c;
    y[n2][3] = d;
  }
  y[1][1] = w16<1, INV>(y[1][1]);
  y[1][2] = w16<2, INV>(y[1][2]);
  y[1][3] = w16<3, INV>(y[1][3]);
  y[2][1] = w16<2, INV>(y[2][1]);
  y[2][2] = w16<4, INV>(y[2][2]);
  y[2][3] = w16<6, INV>(y[2][3]);
  y[3][1] = w16<3, INV>(y[3][1]);
  y[3][2] = w16<6, INV>(y[3][2]);
  y[3][3] = w16<9, INV>(y[3][3]);
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    C a = y[0][k1], b = y[1][k1], c = y[2][k1], d = y[3][k1];
    dft4<INV>(a, b, c, d);
    v[k1] = a;
    v[k1 + 4] = b;
    v[k1 + 8] = c;
    v[k1 + 12] = d;
  }
}

template <int R, bool INV, typename C> __device__ __forceinline__ void dft_small(C* v) {
  if constexpr (R == 2) dft2<INV>(v);
  else if constexpr (R == 3) dft3<INV>(v);
  else if constexpr (R == 4) dft4<INV>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 8) dft8<INV>(v);
  else dft16<INV>(v);
}

// ---------------------------------------------------------------------------
// compile-time radix plan. With at least 16 elements per thread (r16): radix
// 16 as often as the power of two allows, then one 8, 4 or 2, then the 3s;
// otherwise radix 8 as often as it allows, then one 4 or 2, then the 3s.
// ---------------------------------------------------------------------------
constexpr int ct_exp2(int n) {
  int a = 0;
  while (n > 1 && n % 2 == 0) { n /= 2; ++a; }
  return a;
}
constexpr int ct_exp3(int n) {
  int b = 0;
  while (n > 1 && n % 3 == 0) { n /= 3; ++b; }
  return b;
}
constexpr bool ct_r16(int n, int nt) { return nt >= 1 && n / nt >= 16 && ct_exp2(n) >= 4; }
constexpr int ct_npass(int n, bool r16) {
  const int a = ct_exp2(n), w = r16 ? 4 : 3;
  return a / w + (a % w ? 1 : 0) + ct_exp3(n);
}
constexpr int ct_radix(int n, bool r16, int p) {
  const int a = ct_exp2(n), w = r16 ? 4 : 3, nb = a / w, rem = a % w;
  if (p < nb) return r16 ? 16 : 8;
  p -= nb;
  if (rem) {
    if (p == 0) return 1 << rem;
    p -= 1;
  }
  return 3;
}
constexpr int ct_ns(int n, bool r16, int p) {
  int ns = 1;
  for (int i = 0; i < p; ++i) ns *= ct_radix(n, r16, i);
  return ns;
}
constexpr int ct_bt(int n, int nt, bool r16, int p) { return (n / ct_radix(n, r16, p) + nt - 1) / nt; }
constexpr int ct_vmax(int n, int nt, bool r16) {
  int m = 0;
  for (int p = 0; p < ct_npass(n, r16); ++p) {
    const int x = ct_bt(n, nt, r16, p) * ct_radix(n, r16, p);
    m = x > m ? x : m;
  }
  return m;
}

// threads per compile-time transform: ct_threads / ct_threads_y (shared
// with the host, in monc_types.h)
constexpr int ct_threads(int n) { return ct_threads_x_n(n); }
constexpr int ct_threads_y(int n, int ept) { return ct_threads_y_n(n, ept); }

// LDS index of element i of an x-direction transform of length N (bank
// rows permuted by XOR, or padded; see xlds_len)
template <typename T, int N> __device__ __forceinline__ int xpad(int i) {
  return xlds_index(i, N, 2 * (int)sizeof(T));
}

// Compile-time Stockham transform. Thread q (0 <= q < NT) owns butterflies
// b = q + t NT of every pass. Pass p (radix R, Ns = product of the earlier
// radices) reads x[b + r N/R] and writes x[(b - b mod Ns) R + b mod Ns + r Ns]
// after the twiddle W_N^((b mod Ns) r N/(Ns R)); the last pass's outputs are
// x[b + r N/R] again.
template <typename T, int N, int NT, bool INV>
struct CtFft {
  static constexpr bool R16 = ct_r16(N, NT);
  static constexpr int NP = ct_npass(N, R16);
  static constexpr int VMAX = ct_vmax(N, NT, R16);

  template <int P> static constexpr int R() { return ct_radix(N, R16, P); }
  template <int P> static constexpr int NB() { return N / ct_radix(N, R16, P); }
  template <int P> static constexpr int BT() { return ct_bt(N, NT, R16, P); }
  template <int P> __device__ static __forceinline__ bool valid(int b) {
    return (NB<P>() % NT == 0) || b < NB<P>();
  }

  // element index of value v[t R + r] at the input of pass P
  template <int P> __device__ static __forceinline__ int in_index(int q, int t, int r) {
    return q + t * NT + r * NB<P>();
  }

  // tw(i) returns the twiddle exp(-2 pi i i/N) (a global table, or a copy
  // of it in LDS)
  template <int P, class Tw>
  __device__ static __forceinline__ void butterflies(cx<T>* v, int q, const Tw& tw) {
    constexpr int Rr = R<P>(), NS = ct_ns(N, R16, P), TSTEP = N / (NS * Rr);
#pragma unroll
    for (int t = 0; t < BT<P>(); ++t) {
      const int b = q + t * NT;
      if (valid<P>(b)) {
        if constexpr (NS > 1) {
          const int kk = b % NS;
#pragma unroll
          for (int r = 1; r < Rr; ++r) {
            const cx<T> w = tw(kk * r * TSTEP);
            v[t * Rr + r] = INV ? cmulconj(v[t * Rr + r], w) : cmul(v[t * Rr + r], w);
          }
        }
        dft_small<Rr, INV>(v + t * Rr);
      }
    }
  }

  // outputs of pass P -> LDS -> inputs of pass P + 1
  template <int P, class Idx>
  __device__ static __forceinline__ void exchange(cx<T>* v, cx<T>* lds, const Idx& li, int q) {
    constexpr int Rr = R<P>(), NS = ct_ns(N, R16, P);
#pragma unroll
    for (int t = 0; t < BT<P>(); ++t) {
      const int b = q + t * NT;
      if (valid<P>(b)) {
        const int kk = b % NS;
        const int d0 = (b - kk) * Rr + kk;
#pragma unroll
        for (int r = 0; r < Rr; ++r) lds[li(d0 + r * NS)] = v[t * Rr + r];
      }
    }
    __syncthreads();
    constexpr int R2 = R<P + 1>();
#pragma unroll
    for (int t = 0; t < BT<P + 1>(); ++t) {
      const int b = q + t * NT;
      if (valid<P + 1>(b)) {
#pragma unroll
        for (int r = 0; r < R2; ++r) v[t * R2 + r] = lds[li(b + r * NB<P + 1>())];
      }
    }
    __syncthreads();
  }

  template <int P, class Idx, class Tw>
  __device__ static __forceinline__ void run_from(cx<T>* v, cx<T>* lds, const Idx& li, int q, const Tw& tw) {
    butterflies<P>(v, q, tw);
    if constexpr (P + 1 < NP) {
      exchange<P>(v, lds, li, q);
      run_from<P + 1>(v, lds, li, q, tw);
    }
  }

  // Whole transform: v holds the inputs of pass 0 on entry and the outputs of
  // the last pass on exit (positions given by in_index<0> / out_index).
  // Twiddles from the global table tw.
  template <class Idx>
  __device__ static __forceinline__ void run(cx<T>* v, cx<T>* lds, const Idx& li, int q,
                                             const cx<T>* __restrict__ tw) {
    run_from<0>(v, lds, li, q, [tw](int i) { return load_tw(tw + i); });
  }
  // Twiddles from an accessor (e.g. an LDS copy of the table)
  template <class Idx, class Tw>
  __device__ static __forceinline__ void run_tw(cx<T>* v, cx<T>* lds, const Idx& li, int q, const Tw& tw) {
    run_from<0>(v, lds, li, q, tw);
  }

  static constexpr int RL = ct_radix(N, R16, NP - 1);
  static constexpr int BTL = ct_bt(N, NT, R16, NP - 1);
  static constexpr int NBL = N / ct_radix(N, R16, NP - 1);
  __device__ static __forceinline__ bool valid_last(int b) { return (NBL % NT == 0) || b < NBL; }
  // element index of value v[t RL + r] at the output of the last pass
  __device__ static __forceinline__ int out_index(int q, int t, int r) { return q + t * NT + r * NBL; }

  static constexpr int R0 = ct_radix(N, R16, 0);
  static constexpr int BT0 = ct_bt(N, NT, R16, 0);
  static constexpr int NB0 = N / ct_radix(N, R16, 0);
  __device__ static __forceinline__ bool valid_first(int b) { return (NB0 % NT == 0) || b < NB0; }
};

// ---------------------------------------------------------------------------
// runtime-length Stockham pass, in place in LDS (fallback engine)
// ---------------------------------------------------------------------------
template <typename T, int R, bool INV>
__device__ __forceinline__ void stockham_pass(cx<T>* buf, int stride, int N, int Ns,
                                              const cx<T>* __restrict__ tw, int q, int nt) {
  constexpr int BM = (kGenericElems + R - 1) / R;
  const int nb = N / R;
  const int tstep = N / (Ns * R);
  cx<T> v[BM * R];
#pragma unroll
  for (int t = 0; t < BM; ++t) {
    const int b = q + t * nt;
    if (b < nb) {
      const int kk = b % Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) v[t * R + r] = buf[(b + r * nb) * stride];
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const cx<T> w = load_tw(tw + kk * r * tstep);
          v[t * R + r] = INV ? cmulconj(v[t * R + r], w) : cmul(v[t * R + r], w);
        }
      }
      dft_small<R, INV>(v + t * R);
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < BM; ++t) {
    const int b = q + t * nt;
    if (b < nb) {
      const int kk = b % Ns;
      const int dst = (b - kk) * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[(dst + r * Ns) * stride] = v[t * R + r];
    }
  }
  __syncthreads();
}

// Whole runtime-length transform in LDS; every thread of the workgroup must
// call it (barriers).
template <typename T, bool INV>
__device__ __noinline__ void fft_lds(cx<T>* buf, int stride, const FftPlan& fp, const cx<T>* __restrict__ tw,
                                     int q) {
  const int N = fp.n, nt = fp.nt, np = fp.npass;
  int Ns = 1;
  for (int p = 0; p < np; ++p) {
    const int R = fp.rad[p];
    if (R == 8) stockham_pass<T, 8, INV>(buf, stride, N, Ns, tw, q, nt);
    else if (R == 4) stockham_pass<T, 4, INV>(buf, stride, N, Ns, tw, q, nt);
    else if (R == 2) stockham_pass<T, 2, INV>(buf, stride, N, Ns, tw, q, nt);
    else stockham_pass<T, 3, INV>(buf, stride, N, Ns, tw, q, nt);
    Ns *= R;
  }
}

}  // namespace monc

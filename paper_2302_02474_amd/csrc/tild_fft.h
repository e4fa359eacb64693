// Batched complex FFTs of lines held in LDS, for lengths that are products of
// 2, 3 and 5 (radix 8, 4, 2, 3, 5 passes).  Each pass is a Stockham
// autosort pass: butterfly j of a line reads elements j + r*n/R, multiplies by
// the twiddles w^(r*(j mod s)) with w = exp(-+2 pi i/(s R)), applies a
// radix-R DFT and writes elements (j - j mod s)*R + j mod s + r*s, where s is
// the product of the radices already applied.  After the last pass the line
// is in natural order.  Every pass reads all of its inputs into registers
// before a barrier and writes after it, so passes run in place.
#pragma once

#include "tild_common.h"

namespace tild {

constexpr int kMaxRadixStages = 16;

// Factorisation of one transform length and the offset of its twiddle table
// (exp(-2 pi i m/n), m = 0..n-1) inside the context's twiddle array.
struct FftPlan {
    int n;
    int nst;
    int tw;
    int radix[kMaxRadixStages];
};

// Which LDS elements form the lines: line l starts at
// (l % l1) * s1 + (l / l1) * s2 and its elements are `es` apart.
struct LineMap {
    int lines, l1, s1, s2, es;
};

// Elements each thread may hold in registers during one pass.
constexpr int kFftRegElems = 32;

// Radix kernels.  INV = 0: exp(-2 pi i jk/R); INV = 1: exp(+2 pi i jk/R).
template <int INV, typename C> __device__ __forceinline__ void dft2(C* a) {
    const C t = a[0];
    a[0] = cadd(t, a[1]);
    a[1] = csub(t, a[1]);
}

template <int INV, typename C> __device__ __forceinline__ void dft4(C* a) {
    const C t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    const C t2 = cadd(a[1], a[3]);
    const C d = csub(a[1], a[3]);
    const C t3 = INV ? mul_pi(d) : mul_mi(d);
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
}

template <int INV, typename C> __device__ __forceinline__ void dft8(C* a) {
    using T = decltype(a[0].x);
    C e[4] = {a[0], a[2], a[4], a[6]};
    C o[4] = {a[1], a[3], a[5], a[7]};
    dft4<INV>(e);
    dft4<INV>(o);
    const T r = (T)0.70710678118654752440;
    // w^k o_k, w = exp(-+ 2 pi i / 8)
    const C o1 = INV ? C{r * (o[1].x - o[1].y), r * (o[1].x + o[1].y)}
                     : C{r * (o[1].x + o[1].y), r * (o[1].y - o[1].x)};
    const C o2 = INV ? mul_pi(o[2]) : mul_mi(o[2]);
    const C o3 = INV ? C{-r * (o[3].x + o[3].y), r * (o[3].x - o[3].y)}
                     : C{r * (o[3].y - o[3].x), -r * (o[3].x + o[3].y)};
    a[0] = cadd(e[0], o[0]);
    a[4] = csub(e[0], o[0]);
    a[1] = cadd(e[1], o1);
    a[5] = csub(e[1], o1);
    a[2] = cadd(e[2], o2);
    a[6] = csub(e[2], o2);
    a[3] = cadd(e[3], o3);
    a[7] = csub(e[3], o3);
}

template <int INV, typename C> __device__ __forceinline__ void dft3(C* a) {
    using T = decltype(a[0].x);
    const T h = (T)0.86602540378443864676;  // sin(2 pi / 3)
    const C s = cadd(a[1], a[2]);
    const C d = csub(a[1], a[2]);
    const C y0 = cadd(a[0], s);
    const C t = C{a[0].x - (T)0.5 * s.x, a[0].y - (T)0.5 * s.y};
    const C u = INV ? mul_pi(cscale(d, h)) : mul_mi(cscale(d, h));
    a[0] = y0;
    a[1] = cadd(t, u);
    a[2] = csub(t, u);
}

template <int INV, typename C> __device__ __forceinline__ void dft5(C* a) {
    using T = decltype(a[0].x);
    const T c1 = (T)0.30901699437494742410, c2 = (T)-0.80901699437494742410;
    const T s1 = (T)0.95105651629515357212, s2 = (T)0.58778525229247312917;
    const C b1 = cadd(a[1], a[4]), b2 = cadd(a[2], a[3]);
    const C d1 = csub(a[1], a[4]), d2 = csub(a[2], a[3]);
    const C y0 = cadd(a[0], cadd(b1, b2));
    const C t1 = C{a[0].x + c1 * b1.x + c2 * b2.x, a[0].y + c1 * b1.y + c2 * b2.y};
    const C t2 = C{a[0].x + c2 * b1.x + c1 * b2.x, a[0].y + c2 * b1.y + c1 * b2.y};
    const C u1 = C{s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y};
    const C u2 = C{s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y};
    const C iu1 = INV ? mul_pi(u1) : mul_mi(u1);
    const C iu2 = INV ? mul_pi(u2) : mul_mi(u2);
    a[0] = y0;
    a[1] = cadd(t1, iu1);
    a[4] = csub(t1, iu1);
    a[2] = cadd(t2, iu2);
    a[3] = csub(t2, iu2);
}

template <int R, int INV, typename C> __device__ __forceinline__ void dft_r(C* a) {
    if constexpr (R == 2) dft2<INV>(a);
    else if constexpr (R == 3) dft3<INV>(a);
    else if constexpr (R == 4) dft4<INV>(a);
    else if constexpr (R == 5) dft5<INV>(a);
    else dft8<INV>(a);
}

template <typename C, int R, int INV>
__device__ void fft_pass(C* buf, const LineMap lm, const int n, const int s, const C* __restrict__ tw, const int tid,
                         const int nthr) {
    constexpr int MAXB = kFftRegElems / R;
    const int bpl = n / R;
    const int total = lm.lines * bpl;
    const int tstride = n / (s * R);
    C v[MAXB][R];
    int obase[MAXB];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        const int id = tid + b * nthr;
        obase[b] = -1;
        if (id < total) {
            const int line = id / bpl;
            const int j = id - line * bpl;
            const int base = (line % lm.l1) * lm.s1 + (line / lm.l1) * lm.s2;
            const int k = j % s;
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = buf[base + (j + r * bpl) * lm.es];
            if (s > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    C w = tw[k * r * tstride];
                    if (INV) w.y = -w.y;
                    v[b][r] = cmul(v[b][r], w);
                }
            }
            obase[b] = base + ((j - k) * R + k) * lm.es;
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        if (obase[b] >= 0) {
            dft_r<R, INV>(v[b]);
#pragma unroll
            for (int r = 0; r < R; ++r) buf[obase[b] + r * s * lm.es] = v[b][r];
        }
    }
    __syncthreads();
}

// Transform every line described by `lm` in place.  Requires
// lm.lines * plan.n <= 30 * nthr (checked on the host) and a preceding barrier.
template <typename C, int INV>
__device__ void fft_lines(C* buf, const LineMap lm, const FftPlan& plan, const C* __restrict__ twiddles, int tid,
                          int nthr) {
    const C* tw = twiddles + plan.tw;
    int s = 1;
    for (int st = 0; st < plan.nst; ++st) {
        const int R = plan.radix[st];
        switch (R) {
            case 8: fft_pass<C, 8, INV>(buf, lm, plan.n, s, tw, tid, nthr); break;
            case 4: fft_pass<C, 4, INV>(buf, lm, plan.n, s, tw, tid, nthr); break;
            case 2: fft_pass<C, 2, INV>(buf, lm, plan.n, s, tw, tid, nthr); break;
            case 3: fft_pass<C, 3, INV>(buf, lm, plan.n, s, tw, tid, nthr); break;
            default: fft_pass<C, 5, INV>(buf, lm, plan.n, s, tw, tid, nthr); break;
        }
        s *= R;
    }
}

}  // namespace tild

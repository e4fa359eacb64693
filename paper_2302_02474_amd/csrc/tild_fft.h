// Complex FFTs of lines held in LDS, for lengths that are products of 2, 3
// and 5 (radix 8, 4, 2, 3 and 5 passes).
//
// Each line is owned by a group of G lanes of one wavefront (G divides 64),
// so the passes of a line synchronise at wavefront scope only.  A pass is a
// Stockham autosort pass: butterfly j reads elements j + r*n/R, multiplies
// them by w^(r*(j mod s)) with w = exp(-+2 pi i/(s R)), applies a radix-R DFT
// and writes elements (j - j mod s)*R + j mod s + r*s, s being the product of
// the radices already applied; after the last pass the line is in natural
// order.  A lane holds at most kFftRegElems elements of a pass in registers,
// all loads of a pass precede its stores, so passes run in place.
#pragma once

#include "tild_common.h"

namespace tild {

constexpr int kMaxRadixStages = 8;  // 4-bit radix codes in one 32-bit word
constexpr int kFftRegElems = 8;
constexpr int kPairItems = 16;  // row-pair (un)packing items per lane of an x line

// Factorisation of one transform length, the offset of its twiddle table
// (exp(-2 pi i m/n), m = 0..n-1) inside the context's twiddle array, and the
// lanes per line.
struct FftPlan {
    int n;
    int nst;
    int tw;
    int group;  // lanes per line: a power of two <= 64
    uint32_t codes;  // radix of pass st in bits 4 st .. 4 st + 3
    int r1;     // two-pass transform n = r1 r2 (line_fft2) when > 0, else the radix passes
    int tw2;    // offset of its table w^(l k1), l < r2, k1 < r1, stored [l][k1] with row pitch r1 + 1
    __host__ __device__ __forceinline__ int radix(int st) const { return (int)((codes >> (4 * st)) & 15u); }
};

// Which LDS elements form the lines: line l starts at
// (l % l1) * s1 + (l / l1) * s2 and its elements are `es` apart.  With a
// non-zero swizzle mask (lines of one column each: s1 = 1, s2 = 0), element e
// of line l sits in column l ^ ((e >> 3) & swz) instead of l: the eight
// outputs of a radix-8 butterfly, written to consecutive elements, then fall
// into different LDS banks.
struct LineMap {
    int lines, l1, s1, s2, es, swz;
};

// LDS index of element e of the line starting at `base`.
template <bool SWZ>
__device__ __forceinline__ int line_index(int base, int e, int es, int swz) {
    if constexpr (SWZ) return (base ^ ((e >> 3) & swz)) + e * es;
    else return base + e * es;
}

// Order LDS traffic of the lanes of one wavefront.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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

// 16 points as 4 x 4: transforms of the four residue classes n1 (elements
// n1, n1 + 4, n1 + 8, n1 + 12), the twiddles w16^(n1 k1), then transforms over
// n1; output k1 + 4 k2 in natural order.
template <int INV, typename C> __device__ __forceinline__ void dft16(C* a) {
    using T = decltype(a[0].x);
    C b[4][4];
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) {
        C t[4] = {a[n1], a[n1 + 4], a[n1 + 8], a[n1 + 12]};
        dft4<INV>(t);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) b[n1][k1] = t[k1];
    }
    const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173, r = (T)0.70710678118654752440;
    // w16^e for e = n1 k1 in {1, 2, 3, 4, 6, 9}: (cos, -+sin)(2 pi e / 16)
    auto tw = [&](C v, int e) -> C {
        T wr, wi;
        switch (e) {
            case 1: wr = c1; wi = -s1; break;
            case 2: wr = r; wi = -r; break;
            case 3: wr = s1; wi = -c1; break;
            case 6: wr = -r; wi = -r; break;
            default: wr = -c1; wi = s1; break;  // 9
        }
        if (INV) wi = -wi;
        return C{v.x * wr - v.y * wi, v.x * wi + v.y * wr};
    };
#pragma unroll
    for (int n1 = 1; n1 < 4; ++n1)
#pragma unroll
        for (int k1 = 1; k1 < 4; ++k1) {
            const int e = n1 * k1;
            if (e == 4) b[n1][k1] = INV ? mul_pi(b[n1][k1]) : mul_mi(b[n1][k1]);
            else b[n1][k1] = tw(b[n1][k1], e);
        }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        C t[4] = {b[0][k1], b[1][k1], b[2][k1], b[3][k1]};
        dft4<INV>(t);
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = t[k2];
    }
}

template <int R, int INV, typename C> __device__ __forceinline__ void dft_r(C* a) {
    if constexpr (R == 2) dft2<INV>(a);
    else if constexpr (R == 3) dft3<INV>(a);
    else if constexpr (R == 4) dft4<INV>(a);
    else if constexpr (R == 5) dft5<INV>(a);
    else if constexpr (R == 16) dft16<INV>(a);
    else dft8<INV>(a);
}

// One radix-R pass of the line at `base` by lane `lane` of its group of G.
template <typename C, int R, int INV, bool SWZ>
__device__ __forceinline__ void line_pass(C* buf, const int base, const int es, const int swz, const int n,
                                          const int s, const C* __restrict__ tw, const int lane, const int G) {
    constexpr int MAXB = kFftRegElems / R;
    const int bpl = n / R;
    const int tstride = n / (s * R);
    C v[MAXB][R];
    int ob[MAXB];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        const int j = lane + b * G;
        ob[b] = -1;
        if (j < bpl) {
            const int k = j % s;
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = buf[line_index<SWZ>(base, j + r * bpl, es, swz)];
            if (s > 1) {
                // w^r for r < R from two table reads (w, w^2) and at most three products
                C w[R];
                w[1] = tw[k * tstride];
                if (INV) w[1].y = -w[1].y;
                if constexpr (R > 2) {
                    w[2] = tw[2 * k * tstride];
                    if (INV) w[2].y = -w[2].y;
                }
                if constexpr (R > 3) w[3] = cmul(w[1], w[2]);
                if constexpr (R > 4) w[4] = cmul(w[2], w[2]);
                if constexpr (R > 5) {
                    w[5] = cmul(w[1], w[4]);
                    w[6] = cmul(w[2], w[4]);
                    w[7] = cmul(w[3], w[4]);
                }
#pragma unroll
                for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], w[r]);
            }
            ob[b] = (j - k) * R + k;  // first output element
        }
    }
    wave_sync();
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
        if (ob[b] >= 0) {
            dft_r<R, INV>(v[b]);
#pragma unroll
            for (int r = 0; r < R; ++r) buf[line_index<SWZ>(base, ob[b] + r * s, es, swz)] = v[b][r];
        }
    }
    wave_sync();
}

// The passes of a power-of-two length N with groups of N/8 lanes (the
// group the host picks for these lengths), starting at the pass whose
// already-applied radix product is S: radix 8 while at least 8 elements
// per butterfly remain, then 4 or 2, as the host's plan orders them.  Every
// length, stride and radix is a compile-time constant here, so the index
// arithmetic reduces to shifts, masks and immediate LDS offsets; the
// arithmetic on the elements is that of line_pass.
template <typename C, int INV, bool SWZ, int N, int S>
__device__ __forceinline__ void line_passes_fixed(C* buf, const int base, const int es, const int swz,
                                                  const C* __restrict__ tw, const int lane) {
    if constexpr (S < N) {
        constexpr int R = N / S >= 8 ? 8 : N / S;
        constexpr int G = N / 8, BPL = N / R, NB = BPL / G, TS = N / (S * R);
        static_assert(NB * G == BPL && NB * R <= kFftRegElems, "fixed pass does not fit the lane budget");
        // the lane index made opaque to the optimiser: every address and twiddle
        // derived from it would otherwise be hoisted out of the callers' line
        // loops and held in registers for the whole kernel
        int ln = lane;
        asm volatile("" : "+v"(ln));
        C v[NB][R];
        int ob[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = ln + b * G;
            const int k = j & (S - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = buf[line_index<SWZ>(base, j + r * BPL, es, swz)];
            if constexpr (S > 1) {
                C w[R];
                w[1] = tw[k * TS];
                if (INV) w[1].y = -w[1].y;
                if constexpr (R > 2) {
                    w[2] = tw[2 * k * TS];
                    if (INV) w[2].y = -w[2].y;
                }
                if constexpr (R > 3) w[3] = cmul(w[1], w[2]);
                if constexpr (R > 4) w[4] = cmul(w[2], w[2]);
                if constexpr (R > 5) {
                    w[5] = cmul(w[1], w[4]);
                    w[6] = cmul(w[2], w[4]);
                    w[7] = cmul(w[3], w[4]);
                }
#pragma unroll
                for (int r = 1; r < R; ++r) v[b][r] = cmul(v[b][r], w[r]);
            }
            ob[b] = (j - k) * R + k;
        }
        wave_sync();
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            dft_r<R, INV>(v[b]);
#pragma unroll
            for (int r = 0; r < R; ++r) buf[line_index<SWZ>(base, ob[b] + r * S, es, swz)] = v[b][r];
        }
        wave_sync();
        line_passes_fixed<C, INV, SWZ, N, S * R>(buf, base, es, swz, tw, lane);
    }
}

// Two-pass transform of a line of N = R1 R2 points by G lanes (N / G
// elements each, G dividing R1 and R2), from n = l + R2 m and
// k = k1 + R1 k2:
//   X[k1 + R1 k2] = sum_l w_N^(l k1) w_R2^(l k2) sum_m x[l + R2 m] w_R1^(m k1).
// Pass A: each lane takes R2/G values of l, transforms over m in registers,
// multiplies by w_N^(l k1) (table tw2[l (R1 + 1) + k1]: the padded pitch puts
// the rows the lanes of a group read in different LDS banks) and writes the
// result to element k1 R2 + l -- the elements it read, so no other lane is
// disturbed.  Pass B: each lane takes R1/G values of k1, reads elements
// k1 R2 + l, transforms over l and writes element k1 + R1 k2 (natural
// order).  Two rounds of LDS traffic instead of one per radix pass.
//
// XP: the intermediate element (k1, l) is stored at k1 R2 + (l xor (k1 mod
// R2)) instead, a permutation within each group of R2 that spreads the reads
// of pass B (R2 elements of one k1 per lane) over the LDS banks when lines
// are rows of the plane layout; the line's input and output stay in natural
// order.
template <typename C, int INV, bool SWZ, int N, int R1, int R2, int G, bool XP>
__device__ __forceinline__ void line_fft2(C* buf, const int base, const int es, const int swz,
                                          const C* __restrict__ tw2, const int lane) {
    static_assert(R1 * R2 == N && R1 % G == 0 && R2 % G == 0, "two-pass shape");
    constexpr int NA = R2 / G, NB = R1 / G;
    auto mid = [](int k1, int l) { return k1 * R2 + (XP ? (l ^ (k1 & (R2 - 1))) : l); };
    // the lane index made opaque to the optimiser (see line_passes_fixed)
    int ln = lane;
    asm volatile("" : "+v"(ln));
    {
        C v[NA][R1];
#pragma unroll
        for (int d = 0; d < NA; ++d) {
            const int l = ln + d * G;
#pragma unroll
            for (int m = 0; m < R1; ++m) v[d][m] = buf[line_index<SWZ>(base, l + R2 * m, es, swz)];
        }
#pragma unroll
        for (int d = 0; d < NA; ++d) {
            const int l = ln + d * G;
            dft_r<R1, INV>(v[d]);
            const C* w = tw2 + l * (R1 + 1);
#pragma unroll
            for (int k1 = 1; k1 < R1; ++k1) {
                C wk = w[k1];
                if (INV) wk.y = -wk.y;
                v[d][k1] = cmul(v[d][k1], wk);
            }
#pragma unroll
            for (int k1 = 0; k1 < R1; ++k1) buf[line_index<SWZ>(base, mid(k1, l), es, swz)] = v[d][k1];
        }
    }
    wave_sync();
    {
        C v[NB][R2];
#pragma unroll
        for (int d = 0; d < NB; ++d) {
            const int k1 = ln + d * G;
#pragma unroll
            for (int l = 0; l < R2; ++l) v[d][l] = buf[line_index<SWZ>(base, mid(k1, l), es, swz)];
        }
        wave_sync();
#pragma unroll
        for (int d = 0; d < NB; ++d) {
            const int k1 = ln + d * G;
            dft_r<R2, INV>(v[d]);
#pragma unroll
            for (int k2 = 0; k2 < R2; ++k2) buf[line_index<SWZ>(base, k1 + R1 * k2, es, swz)] = v[d][k2];
        }
    }
    wave_sync();
}

// Transform the line at `base` (elements `es` apart, swizzled with mask swz
// when SWZ) in place; called by all G lanes of the owning group.  XP selects
// the permuted intermediate order of the two-pass shapes (line_fft2).
template <typename C, int INV, bool SWZ = false, bool XP = false>
__device__ __forceinline__ void fft_line(C* buf, const int base, const int es, const FftPlan plan,
                                         const C* __restrict__ twiddles, const int lane, const int swz = 0) {
    const C* tw = twiddles + plan.tw;
    const int G = plan.group;
    if (plan.r1) {
        const C* tw2 = twiddles + plan.tw2;
        switch (plan.n) {
            case 64: line_fft2<C, INV, SWZ, 64, 8, 8, 8, XP>(buf, base, es, swz, tw2, lane); return;
            case 128: line_fft2<C, INV, SWZ, 128, 16, 8, 8, XP>(buf, base, es, swz, tw2, lane); return;
            case 256: line_fft2<C, INV, SWZ, 256, 16, 16, 16, XP>(buf, base, es, swz, tw2, lane); return;
            default: break;
        }
    }
    if (G * 8 == plan.n) {
        switch (plan.n) {
            case 16: line_passes_fixed<C, INV, SWZ, 16, 1>(buf, base, es, swz, tw, lane); return;
            case 32: line_passes_fixed<C, INV, SWZ, 32, 1>(buf, base, es, swz, tw, lane); return;
            case 64: line_passes_fixed<C, INV, SWZ, 64, 1>(buf, base, es, swz, tw, lane); return;
            case 128: line_passes_fixed<C, INV, SWZ, 128, 1>(buf, base, es, swz, tw, lane); return;
            case 256: line_passes_fixed<C, INV, SWZ, 256, 1>(buf, base, es, swz, tw, lane); return;
            default: break;
        }
    }
    int s = 1;
    for (int st = 0; st < plan.nst; ++st) {
        const int R = plan.radix(st);
        switch (R) {
            case 8: line_pass<C, 8, INV, SWZ>(buf, base, es, swz, plan.n, s, tw, lane, G); break;
            case 4: line_pass<C, 4, INV, SWZ>(buf, base, es, swz, plan.n, s, tw, lane, G); break;
            case 2: line_pass<C, 2, INV, SWZ>(buf, base, es, swz, plan.n, s, tw, lane, G); break;
            case 3: line_pass<C, 3, INV, SWZ>(buf, base, es, swz, plan.n, s, tw, lane, G); break;
            default: line_pass<C, 5, INV, SWZ>(buf, base, es, swz, plan.n, s, tw, lane, G); break;
        }
        s *= R;
    }
}

// Transform every line of `lm` with the block's threads split into groups of
// plan.group lanes.  Needs a block barrier before (inputs written by other
// waves) and, if other waves read the result, after.
template <typename C, int INV, bool SWZ = false, bool XP = false>
__device__ __forceinline__ void fft_lines(C* buf, const LineMap lm, const FftPlan plan, const C* __restrict__ twiddles,
                                          int tid, int nthr) {
    const int G = plan.group;
    const int lane = tid % G, grp = tid / G, ngrp = nthr / G;
    // line l = q l1 + r, stepped by ngrp = dq l1 + dr without a division per line
    const int dq = ngrp / lm.l1, dr = ngrp % lm.l1;
    int q = grp / lm.l1, r = grp % lm.l1;
    for (int l = grp; l < lm.lines; l += ngrp) {
        fft_line<C, INV, SWZ, XP>(buf, r * lm.s1 + q * lm.s2, lm.es, plan, twiddles, lane, lm.swz);
        q += dq;
        r += dr;
        if (r >= lm.l1) {
            r -= lm.l1;
            ++q;
        }
    }
}

}  // namespace tild

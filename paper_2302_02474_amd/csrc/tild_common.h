// Device-side helpers shared by the TILD kernels: complex arithmetic, grid
// geometry, fixed-point positions, B-spline assignment weights and the Philox
// noise generator.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tild {

template <typename T> struct CplxOf;
template <> struct CplxOf<float> { using type = float2; };
template <> struct CplxOf<double> { using type = double2; };
template <typename T> using cplx = typename CplxOf<T>::type;

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
    return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
    return C{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename C, typename T> __device__ __forceinline__ C cscale(C a, T s) { return C{a.x * s, a.y * s}; }
// -i * a and +i * a
template <typename C> __device__ __forceinline__ C mul_mi(C a) { return C{a.y, -a.x}; }
template <typename C> __device__ __forceinline__ C mul_pi(C a) { return C{-a.y, a.x}; }

// Grid geometry.  Real grids are stored [z][y][x] (x fastest); half spectra
// (real-to-complex along x) are stored [z][ky][kx] with hx = mx/2 + 1.
struct Dims {
    int mx, my, mz;  // grid points
    int hx;          // mx/2 + 1
    int npair;       // (my + 1) / 2: row pairs packed into one complex row
    int hxp;         // LDS half-row pitch: >= hx and 2 hxp >= mx + P - 1 (4 mod 16 with a two-pass x transform, else odd)
    int npg;         // LDS row pairs including ghost rows: ceil((my + P - 1) / 2)
    int ylines;      // y transforms per plane: hx, or hx - 1 when the kx = 0 and mx/2 columns share one
    int swc;         // columns kx < swc of an LDS half spectrum are swizzled (ylines or 0)
    long long m;     // mx*my*mz
    long long hplane;  // my*hx complex per half-spectrum plane
    double lx, ly, lz;
    int ntw2;        // entries of the two-pass twiddle tables (lengths that use them)
    // complex twiddle entries: exp(-2 pi i m/n) for each axis, then the two-pass tables
    __host__ __device__ __forceinline__ int ntw() const { return mx + my + mz + ntw2; }
};

// The dispatcher hands consecutive workgroups of a launch to the device's 8
// XCDs in turn (linear id mod 8), and each XCD has its own L2.  This maps the
// linear id b of a launch of G workgroups to a logical tile id such that each
// XCD receives one contiguous range of tiles (a bijection of [0, G)): tiles
// that read overlapping data then share one L2.
__device__ __forceinline__ int xcd_contiguous(int b, int G) {
    constexpr int kXcds = 8;
    const int q = G / kXcds, r = G % kXcds, x = b % kXcds, s = b / kXcds;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + s;
}

// Positions are unsigned 32-bit fractions of the box edge: x = q * L / 2^32.
// The grid coordinate u = x / h = q * M / 2^32 is a 64-bit fixed-point number
// with 32 fractional bits, so cell indices and fractional offsets are exact.
//
// Assignment: a bead at u touches the P nodes g0 .. g0+P-1 with
// g0 = floor(u - P/2) + 1, and the node g0+j has weight B_P(u - g0 - j), B_P
// the centred cardinal B-spline of order P.  With f = frac(u - P/2) that
// weight is the uncentred spline M_P(f + P-1-j), where
//   M_1 = 1 on [0,1);  M_k(s) = [s M_{k-1}(s) + (k-s) M_{k-1}(s-1)] / (k-1).
// On [i, i+1), M_P is a polynomial of degree P-1 in f = s - i; its
// coefficients follow from the recursion by polynomial arithmetic and are
// formed at compile time, so a weight costs P-1 fused multiply-adds.
template <int P> struct SplinePieces {
    double c[P][P];  // M_P(f + i) = sum_k c[i][k] f^k, 0 <= f < 1
};

template <int P> constexpr SplinePieces<P> spline_pieces() {
    SplinePieces<P> r{};
    if constexpr (P == 1) {
        r.c[0][0] = 1.0;
    } else {
        const SplinePieces<P - 1> m = spline_pieces<P - 1>();
        for (int i = 0; i < P; ++i)
            for (int k = 0; k < P; ++k) {
                double v = 0.0;
                if (i <= P - 2) {  // (f + i) M_{P-1}(f + i)
                    if (k >= 1) v += m.c[i][k - 1];
                    if (k <= P - 2) v += i * m.c[i][k];
                }
                if (i >= 1) {  // (P - i - f) M_{P-1}(f + i - 1)
                    if (k <= P - 2) v += (P - i) * m.c[i - 1][k];
                    if (k >= 1) v -= m.c[i - 1][k - 1];
                }
                r.c[i][k] = v / (P - 1);
            }
    }
    return r;
}

// Weight of stencil node j (0 <= j < P) at fraction f: M_P(f + P-1-j).
template <typename T, int P, int J> __device__ __forceinline__ T spline_weight(T f) {
    constexpr SplinePieces<P> sp = spline_pieces<P>();
    constexpr int i = P - 1 - J;
    T v = (T)sp.c[i][P - 1];
#pragma unroll
    for (int k = P - 2; k >= 0; --k) v = v * f + (T)sp.c[i][k];
    return v;
}

template <typename T, int P, int J = 0> __device__ __forceinline__ void spline_weights(T f, T w[P]) {
    if constexpr (J < P) {
        w[J] = spline_weight<T, P, J>(f);
        spline_weights<T, P, J + 1>(f, w);
    }
}

// Derivative dw_j/df of the weight of node j (P >= 2): the derivative of the
// same polynomial piece, with compile-time coefficients k c[i][k].
template <typename T, int P, int J> __device__ __forceinline__ T spline_dweight(T f) {
    constexpr SplinePieces<P> sp = spline_pieces<P>();
    constexpr int i = P - 1 - J;
    T v = (T)((P - 1) * sp.c[i][P - 1]);
#pragma unroll
    for (int k = P - 2; k >= 1; --k) v = v * f + (T)(k * sp.c[i][k]);
    return v;
}

template <typename T, int P, int J = 0> __device__ __forceinline__ void spline_dweights(T f, T dw[P]) {
    if constexpr (J < P) {
        dw[J] = spline_dweight<T, P, J>(f);
        spline_dweights<T, P, J + 1>(f, dw);
    }
}

// Second derivative d^2 w_j/df^2 (P >= 3): coefficients k (k - 1) c[i][k].
template <typename T, int P, int J> __device__ __forceinline__ T spline_d2weight(T f) {
    constexpr SplinePieces<P> sp = spline_pieces<P>();
    constexpr int i = P - 1 - J;
    T v = (T)((P - 1) * (P - 2) * sp.c[i][P - 1]);
#pragma unroll
    for (int k = P - 2; k >= 2; --k) v = v * f + (T)(k * (k - 1) * sp.c[i][k]);
    return v;
}

template <typename T, int P, int J = 0> __device__ __forceinline__ void spline_d2weights(T f, T d2w[P]) {
    if constexpr (J < P) {
        d2w[J] = P >= 3 ? spline_d2weight<T, P, J>(f) : (T)0;
        spline_d2weights<T, P, J + 1>(f, d2w);
    }
}

// (u - P/2) * 2^32 for fixed-point q on an axis of m points.
__device__ __forceinline__ int64_t stencil_fixed(uint32_t q, int m, int P) {
    return (int64_t)((uint64_t)q * (uint64_t)(uint32_t)m) - ((int64_t)P << 31);
}

// First stencil node g0 = floor(u - P/2) + 1, wrapped into [0, m).  Before
// wrapping 1 - P/2 <= g0 <= m - P/2 (m only for P = 1, the nearest node of a
// bead just below the upper edge), so with m >= P one add or subtract wraps.
__device__ __forceinline__ int wrap_start(int g, int m, int P) {
    if (P == 1) return g >= m ? g - m : g;
    return g < 0 ? g + m : g;
}

__device__ __forceinline__ int stencil_start(uint32_t q, int m, int P) {
    return wrap_start((int)(stencil_fixed(q, m, P) >> 32) + 1, m, P);
}

// Fraction f = frac(u - P/2) of fixed-point q.
template <typename T> __device__ __forceinline__ T stencil_fraction(uint32_t q, int m, int P) {
    const uint32_t fr = q * (uint32_t)m - ((uint32_t)P << 31);  // low 32 bits, modulo 2^32
    return (T)fr * (T)2.3283064365386963e-10;                  // 2^-32
}

// g0 (wrapped) and the P weights of coordinate q.
template <typename T, int P>
__device__ __forceinline__ void assignment_weights(uint32_t q, int m, int& g0, T w[P]) {
    const int64_t s = stencil_fixed(q, m, P);
    g0 = wrap_start((int)(s >> 32) + 1, m, P);
    const T f = (T)(uint32_t)(s & 0xffffffffLL) * (T)2.3283064365386963e-10;  // 2^-32
    spline_weights<T, P>(f, w);
}

// Grid record of one coordinate, formed once per step when the beads are
// sorted and read by the single-precision spread and interpolation: the
// wrapped first stencil node g0 (< 256) in the top 8 bits and the fraction
// f = frac(u - P/2) truncated to 24 bits below (the precision a float
// fraction holds near 1).
__device__ __forceinline__ uint32_t grid_record(uint32_t q, int m, int P) {
    const int64_t s = stencil_fixed(q, m, P);
    const int g0 = wrap_start((int)(s >> 32) + 1, m, P);
    return ((uint32_t)g0 << 24) | ((uint32_t)s >> 8);
}

// First stencil nodes (x, y) and fractions (x, y, z) of a bead: from its grid
// record when T is float (sx, sy, sz unused), from its fixed-point position
// minus the shift when T is double.
template <typename T> struct BeadFrac {
    int gx, gy;
    T fx, fy, fz;
};
template <typename T, int P>
__device__ __forceinline__ BeadFrac<T> bead_frac(const uint4 q, uint32_t sx, uint32_t sy, uint32_t sz, int mx, int my,
                                                 int mz) {
    BeadFrac<T> b;
    if constexpr (sizeof(T) == 4) {
        constexpr float k24 = 5.9604644775390625e-8f;  // 2^-24
        b.gx = (int)(q.x >> 24);
        b.gy = (int)(q.y >> 24);
        b.fx = (float)(q.x & 0xffffffu) * k24;
        b.fy = (float)(q.y & 0xffffffu) * k24;
        b.fz = (float)(q.z & 0xffffffu) * k24;
    } else {
        b.gx = stencil_start(q.x - sx, mx, P);
        b.gy = stencil_start(q.y - sy, my, P);
        b.fx = stencil_fraction<T>(q.x - sx, mx, P);
        b.fy = stencil_fraction<T>(q.y - sy, my, P);
        b.fz = stencil_fraction<T>(q.z - sz, mz, P);
    }
    return b;
}

// a * b + c rounded once, in T.
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Minimum-image separation (in box units * 2^32) of two fixed-point coordinates.
__device__ __forceinline__ int32_t fixed_delta(uint32_t a, uint32_t b) { return (int32_t)(a - b); }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of
//   (c0, c1, c2, c3) <- (hi(B*c2) ^ c1 ^ k0, lo(B*c2), hi(A*c0) ^ c3 ^ k1, lo(A*c0))
// with the key advanced by the Weyl increments between rounds.
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
    constexpr uint32_t A = 0xD2511F53u, B = 0xCD9E8D57u;
    constexpr uint32_t WA = 0x9E3779B9u, WB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += WA;
            k1 += WB;
        }
        // both halves of each 32 x 32 -> 64-bit product from one multiply
        const uint64_t p0 = (uint64_t)A * c.x, p1 = (uint64_t)B * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    }
    return c;
}

// -2 ln(u) for u = (w + 1/2) 2^-32, accurate also when u is close to 1.
__device__ __forceinline__ float neg2log_u(uint32_t w) {
    if (w >= 0x80000000u) {
        const float tail = ((float)(0xffffffffu - w) + 0.5f) * 2.3283064365386963e-10f;  // 1 - u
        return -2.0f * log1pf(-tail);
    }
    return -2.0f * logf(((float)w + 0.5f) * 2.3283064365386963e-10f);
}
__device__ __forceinline__ double neg2log_u_d(uint32_t w) {
    return -2.0 * log(((double)w + 0.5) * 2.3283064365386963e-10);
}

// Unit Gaussian increments of bead `id` at step `step` (Box-Muller on the
// four Philox words: x, y from words 0, 1 and z from words 2, 3).
template <typename T> struct Noise;
template <> struct Noise<float> {
    __device__ static void draw(uint32_t id, uint64_t step, uint64_t seed, float xi[3]) {
        const U4 r = philox4x32_10(U4{id, (uint32_t)step, (uint32_t)(step >> 32), 0u}, (uint32_t)seed,
                                   (uint32_t)(seed >> 32));
        const float r01 = sqrtf(neg2log_u(r.x));
        const float r23 = sqrtf(neg2log_u(r.z));
        float s1, c1, s3, c3;
        sincospif(2.0f * (((float)r.y + 0.5f) * 2.3283064365386963e-10f), &s1, &c1);
        sincospif(2.0f * (((float)r.w + 0.5f) * 2.3283064365386963e-10f), &s3, &c3);
        xi[0] = r01 * c1;
        xi[1] = r01 * s1;
        xi[2] = r23 * c3;
    }
};
template <> struct Noise<double> {
    __device__ static void draw(uint32_t id, uint64_t step, uint64_t seed, double xi[3]) {
        const U4 r = philox4x32_10(U4{id, (uint32_t)step, (uint32_t)(step >> 32), 0u}, (uint32_t)seed,
                                   (uint32_t)(seed >> 32));
        const double r01 = sqrt(neg2log_u_d(r.x));
        const double r23 = sqrt(neg2log_u_d(r.z));
        double s1, c1, s3, c3;
        sincospi(2.0 * (((double)r.y + 0.5) * 2.3283064365386963e-10), &s1, &c1);
        sincospi(2.0 * (((double)r.w + 0.5) * 2.3283064365386963e-10), &s3, &c3);
        xi[0] = r01 * c1;
        xi[1] = r01 * s1;
        xi[2] = r23 * c3;
    }
};

}  // namespace tild

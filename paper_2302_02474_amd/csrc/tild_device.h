// HIP kernels of the TILD particle-mesh step for gfx950.
//
// Per step (paper, Sec. "Long-range interactions", Eq. PMM and Fig. pmm):
//   spread_xy   per (z-plane, species): the beads whose order-P B-spline
//               stencil reaches the plane are accumulated in LDS (counts minus
//               their mean), then real-to-complex FFT along x, FFT along y
//   z_kmul      per column block: FFT along z, multiply by the smeared
//               chi/kappa kernel, inverse FFT along z of Phi_K and ik_z Phi_K
//   xy_c2r      per (z-plane, species, axis): ik_x or ik_y applied, inverse
//               FFT along y and complex-to-real along x -> one gradient plane
//               in LDS, interpolated onto the beads that reach it with the
//               same weights (one partial force per bead, plane and axis)
//   update      F_i = -sum_g W_i(g) grad phi_{s_i}(g) (the sum of its
//               partials) + bond force, Philox noise, Euler-Maruyama update,
//               each moved bead's bin key and rank
//   bin_scan    bin counts -> bin starts
//   scatter     beads and bond partners into the new sorted order; the noise
//               sums of the next step's centre-of-mass shift
#pragma once

#include "tild_kernels.h"

#include <type_traits>

namespace tild {


constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kTwo32 = 4294967296.0;
constexpr double kInvTwo32 = 2.3283064365386962890625e-10;

// ------------------------------------------------------------ reductions

template <typename V> __device__ __forceinline__ V wave_sum(V v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum NV values over the block; thread 0 receives the totals.
template <typename V, int NV>
__device__ __forceinline__ void block_sum(V* vals, V* scratch /* [NV][nwaves] */, int tid, int nthr) {
    const int lane = tid & 63, wave = tid >> 6, nw = nthr >> 6;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        V s = wave_sum(vals[q]);
        if (lane == 0) scratch[q * nw + wave] = s;
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            V s = 0;
            for (int w = 0; w < nw; ++w) s += scratch[q * nw + w];
            vals[q] = s;
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------ bins

// Bin key of a bead: (species, first stencil plane in z, first stencil row in y).
__device__ __forceinline__ uint32_t bin_key(uint32_t qy, uint32_t qz, uint32_t species, const Dims d, int P) {
    const int gy = stencil_start(qy, d.my, P), gz = stencil_start(qz, d.mz, P);
    return (uint32_t)((species * (uint32_t)d.mz + (uint32_t)gz) * (uint32_t)d.my + (uint32_t)gy);
}

// ------------------------------------------------------------ LDS plane layout
//
// A real plane r[y][x] sits in LDS as complex rows of pitch zp = 2 hxp:
// complex row p holds rows 2p (real parts) and 2p+1 (imaginary parts), so
// r[y][x] is float number pr * (y >> 1) + (y & 1) + 2x, pr = 2 zp.  Columns
// mx .. mx+P-2 and rows my .. my+P-2 are ghosts of columns and rows 0 .. P-2,
// so that a stencil starting at any (g0y, g0x) in [0, my) x [0, mx) is read or
// written without wrapping.  The half spectrum of the same plane keeps row ky
// at complex offset ky * hxp.

// LDS index of half-spectrum element (ky, kx): row pitch hxp; columns
// kx < swc are swizzled within aligned groups of 16 by (ky >> 3) & 15, the
// layout the y transforms use (LineMap swz).
__device__ __forceinline__ int hidx(const Dims d, int ky, int kx) {
    return ky * d.hxp + (kx < d.swc ? kx ^ ((ky >> 3) & 15) : kx);
}

// Float offsets of rows gy .. gy+P-1 (gy in [0, my)).
template <int P> struct RowOffsets {
    int o[P];
    __device__ __forceinline__ RowOffsets(int gy, int pr) {
        const int e = gy & 1;
        const int o0 = __mul24(gy >> 1, pr) + e;
#pragma unroll
        for (int b = 0; b < P; ++b) {
            // rows gy + b: (gy + b) >> 1 = (gy >> 1) + ((e + b) >> 1), parity (e + b) & 1
            const int even = (b >> 1) * pr + (b & 1);                    // e == 0
            const int odd = ((b + 1) >> 1) * pr + ((b + 1) & 1) - 1;     // e == 1
            o[b] = o0 + (e ? odd : even);
        }
    }
};

// Walk (p, x) over a row-major range of pitch w, in steps of n elements.
struct Walk2 {
    int p, x, dp, dx, w;
    __device__ __forceinline__ Walk2(int i0, int w_, int n) : w(w_) {
        p = i0 / w;
        x = i0 - p * w;
        dp = n / w;
        dx = n - dp * w;
    }
    __device__ __forceinline__ void next() {
        p += dp;
        x += dx;
        if (x >= w) {
            x -= w;
            ++p;
        }
    }
};

// ------------------------------------------------------------ spread + xy forward

// Accumulate the counts of every species-K bead whose stencil reaches plane z
// (the beads of the P slabs z-P+1 .. z) into the extended LDS plane (ghost
// cells included) as fixed-point integers, each contribution rounded to a
// multiple of 1/scale: int32 cells in single precision, int64 cells in double
// precision.  Integer LDS atomics are order-independent, so every run gives
// the same bits, and far faster than float ones on this hardware.
//
// pos holds the beads' grid records in single precision, their fixed-point
// positions in double precision (bead_frac).
template <typename T, int P>
__device__ __forceinline__ void spread_plane(unsigned char* __restrict__ lds, const uint4* __restrict__ pos,
                                             const uint32_t* __restrict__ bin_start,
                                             const uint32_t* __restrict__ qs, const Dims d, int z, int K, T scale,
                                             int tid, int nthr) {
    using A = typename std::conditional<sizeof(T) == 4, uint32_t, unsigned long long>::type;
    A* acc = reinterpret_cast<A*>(lds);
    const uint32_t sx = qs[0], sy = qs[1], sz = qs[2];
    const int pr = 4 * d.hxp;
#pragma unroll
    for (int c = 0; c < P; ++c) {
        int s = z - c;
        if (s < 0) s += d.mz;
        const int b0 = (K * d.mz + s) * d.my;
        const uint32_t j0 = bin_start[b0], j1 = bin_start[b0 + d.my];
        // one bead per thread at a time, the next bead's record loaded while
        // this one is spread (see push_plane)
        const uint32_t jt = j0 + (uint32_t)tid;
        if (jt < j1) {
            uint4 qn = pos[jt];
            for (uint32_t j = jt; j < j1; j += (uint32_t)nthr) {
                const uint4 q = qn;
                const uint32_t jn = j + (uint32_t)nthr;
                qn = pos[jn < j1 ? jn : j1 - 1u];
                const BeadFrac<T> bf = bead_frac<T, P>(q, sx, sy, sz, d.mx, d.my, d.mz);
                T wx[P], wy[P];
                spline_weights<T, P>(bf.fx, wx);
                spline_weights<T, P>(bf.fy, wy);
                // the bead's slab is s: its z weight on plane z = s + c is w_c (c is
                // a constant after unrolling, so only that weight is evaluated)
                T wz[P];
                spline_weights<T, P>(bf.fz, wz);
                const T w0 = wz[c] * scale;
                const RowOffsets<P> ro(bf.gy, pr);
                const int gx = bf.gx;
#pragma unroll
                for (int b = 0; b < P; ++b) {
                    A* row = acc + ro.o[b] + 2 * gx;
                    const T wyz = w0 * wy[b];
                    // contributions are >= 0: adding 1/2 and truncating rounds to the nearest multiple
#pragma unroll
                    for (int a = 0; a < P; ++a) {
                        if constexpr (sizeof(T) == 4)
                            atomicAdd(row + 2 * a, __float2uint_rz(fmaf(wyz, wx[a], 0.5f)));
                        else
                            atomicAdd(row + 2 * a, (unsigned long long)__double2ll_rz(fma(wyz, wx[a], 0.5)));
                    }
                }
            }
        }
    }
}

// Directional counts (adjoint and Hessian-vector products): every bead j of
// the P slabs z-P+1 .. z adds grad W_j(g) . v_j to the node g of plane z it
// reaches, accumulated as fixed-point integers (A: int32 cells in single
// precision, int64 in double) at the scale weighted_scale chose from the
// plane's largest |v_x|/h_x + |v_y|/h_y + |v_z|/h_z (a B-spline and its
// derivative are at most 1).  vdir: [n][4] per sorted bead.
template <typename T, int P, typename A>
__device__ __forceinline__ void spread_plane_dir(A* __restrict__ acc, const uint4* __restrict__ pos,
                                                 const uint32_t* __restrict__ bin_start,
                                                 const uint32_t* __restrict__ qs, const Dims d, int z, int K,
                                                 const T* __restrict__ vdir, T scale, int tid, int nthr) {
    const uint32_t sx = qs[0], sy = qs[1], sz = qs[2];
    const int pr = 4 * d.hxp;
    const T ihx = (T)(d.mx / d.lx), ihy = (T)(d.my / d.ly), ihz = (T)(d.mz / d.lz);
#pragma unroll
    for (int c = 0; c < P; ++c) {
        int s = z - c;
        if (s < 0) s += d.mz;
        const int b0 = (K * d.mz + s) * d.my;
        const uint32_t j0 = bin_start[b0], j1 = bin_start[b0 + d.my];
        for (uint32_t j = j0 + (uint32_t)tid; j < j1; j += (uint32_t)nthr) {
            const uint4 q = pos[j];
            const T vx = vdir[4 * (long long)j] * ihx * scale, vy = vdir[4 * (long long)j + 1] * ihy * scale;
            const T vz = vdir[4 * (long long)j + 2] * ihz * scale;
            const BeadFrac<T> bf = bead_frac<T, P>(q, sx, sy, sz, d.mx, d.my, d.mz);
            const int gx = bf.gx;
            T wx[P], wy[P], dwx[P], dwy[P];
            spline_weights<T, P>(bf.fx, wx);
            spline_weights<T, P>(bf.fy, wy);
            spline_dweights<T, P>(bf.fx, dwx);
            spline_dweights<T, P>(bf.fy, dwy);
            const T fz = bf.fz;
            T wzs[P], dwzs[P];  // only entry c survives unrolling
            spline_weights<T, P>(fz, wzs);
            spline_dweights<T, P>(fz, dwzs);
            const RowOffsets<P> ro(bf.gy, pr);
#pragma unroll
            for (int b = 0; b < P; ++b) {
                A* row = acc + ro.o[b] + 2 * gx;
                const T cy = wy[b] * wzs[c] * vx, cr = dwy[b] * wzs[c] * vy + wy[b] * dwzs[c] * vz;
#pragma unroll
                for (int a = 0; a < P; ++a) {
                    if constexpr (sizeof(T) == 4)
                        atomicAdd(row + 2 * a, (A)__float2int_rn(dwx[a] * cy + wx[a] * cr));
                    else
                        atomicAdd(row + 2 * a, (A)__double2ll_rn(dwx[a] * cy + wx[a] * cr));
                }
            }
        }
    }
}

// Largest |v_x| ih_x + |v_y| ih_y + |v_z| ih_z over the beads of the P slabs
// z-P+1 .. z that this thread visits (vdir [n][4]).
template <typename T, int P>
__device__ __forceinline__ T dir_weight_max(const uint32_t* __restrict__ bin_start, const Dims d, int z, int K,
                                            const T* __restrict__ vdir, int tid, int nthr) {
    const T ihx = (T)(d.mx / d.lx), ihy = (T)(d.my / d.ly), ihz = (T)(d.mz / d.lz);
    T m = 0;
#pragma unroll
    for (int c = 0; c < P; ++c) {
        int s = z - c;
        if (s < 0) s += d.mz;
        const int b0 = (K * d.mz + s) * d.my;
        const uint32_t j0 = bin_start[b0], j1 = bin_start[b0 + d.my];
        for (uint32_t j = j0 + (uint32_t)tid; j < j1; j += (uint32_t)nthr) {
            const T v = fabs(vdir[4 * (long long)j]) * ihx + fabs(vdir[4 * (long long)j + 1]) * ihy +
                        fabs(vdir[4 * (long long)j + 2]) * ihz;
            m = v > m ? v : m;
        }
    }
    return m;
}

// Weighted counts (adjoint of the ik route): every bead j of the P slabs
// z-P+1 .. z adds q_j W_j(g), q_j = vdir[4 j + comp], to the node g of plane z
// it reaches, accumulated as fixed-point integers (A: int32 cells in single
// precision, int64 in double) at the scale weighted_scale chose: each
// contribution rounded to the nearest multiple of 1/scale, the sums exact and
// independent of their order.
template <typename T, int P, typename A>
__device__ __forceinline__ void spread_plane_weighted(A* __restrict__ acc, const uint4* __restrict__ pos,
                                                      const uint32_t* __restrict__ bin_start,
                                                      const uint32_t* __restrict__ qs, const Dims d, int z, int K,
                                                      const T* __restrict__ vdir, int comp, T scale, int tid,
                                                      int nthr) {
    const uint32_t sx = qs[0], sy = qs[1], sz = qs[2];
    const int pr = 4 * d.hxp;
#pragma unroll
    for (int c = 0; c < P; ++c) {
        int s = z - c;
        if (s < 0) s += d.mz;
        const int b0 = (K * d.mz + s) * d.my;
        const uint32_t j0 = bin_start[b0], j1 = bin_start[b0 + d.my];
        for (uint32_t j = j0 + (uint32_t)tid; j < j1; j += (uint32_t)nthr) {
            const uint4 q = pos[j];
            const T qj = vdir[4 * (long long)j + comp];
            const BeadFrac<T> bf = bead_frac<T, P>(q, sx, sy, sz, d.mx, d.my, d.mz);
            const int gx = bf.gx;
            T wx[P], wy[P], wzs[P];  // only wzs[c] survives unrolling
            spline_weights<T, P>(bf.fx, wx);
            spline_weights<T, P>(bf.fy, wy);
            spline_weights<T, P>(bf.fz, wzs);
            const RowOffsets<P> ro(bf.gy, pr);
            const T w0 = qj * wzs[c] * scale;
#pragma unroll
            for (int b = 0; b < P; ++b) {
                A* row = acc + ro.o[b] + 2 * gx;
                const T wyz = w0 * wy[b];
#pragma unroll
                for (int a = 0; a < P; ++a) {
                    if constexpr (sizeof(T) == 4)
                        atomicAdd(row + 2 * a, (A)__float2int_rn(wyz * wx[a]));
                    else
                        atomicAdd(row + 2 * a, (A)__double2ll_rn(wyz * wx[a]));
                }
            }
        }
    }
}

// Largest |vdir[4 j + comp]| over the beads of the P slabs z-P+1 .. z that
// this thread visits.
template <typename T, int P>
__device__ __forceinline__ T weight_max(const uint32_t* __restrict__ bin_start, const Dims d, int z, int K,
                                        const T* __restrict__ vdir, int comp, int tid, int nthr) {
    T m = 0;
#pragma unroll
    for (int c = 0; c < P; ++c) {
        int s = z - c;
        if (s < 0) s += d.mz;
        const int b0 = (K * d.mz + s) * d.my;
        const uint32_t j0 = bin_start[b0], j1 = bin_start[b0 + d.my];
        for (uint32_t j = j0 + (uint32_t)tid; j < j1; j += (uint32_t)nthr) {
            const T v = fabs(vdir[4 * (long long)j + comp]);
            m = v > m ? v : m;
        }
    }
    return m;
}

// Add the ghost cells of the extended plane into the cells they alias
// (columns first, over real and ghost rows, then rows).  A: uint32_t or
// unsigned long long (fixed point, wrapping integer sums).  Ends with a barrier.
template <typename A, int P>
__device__ __forceinline__ void fold_ghosts(A* acc, const Dims d, int tid, int nthr) {
    if constexpr (P > 1) {
        const int pr = 4 * d.hxp;
        for (int i = tid; i < (d.my + P - 1) * (P - 1); i += nthr) {
            const int y = i / (P - 1), e = i - y * (P - 1);
            const int o = __mul24(y >> 1, pr) + (y & 1);
            acc[o + 2 * e] += acc[o + 2 * (d.mx + e)];
        }
        __syncthreads();
        for (int i = tid; i < (P - 1) * d.mx; i += nthr) {
            const int e = i / d.mx, x = i - e * d.mx;
            const int yg = d.my + e;
            const int og = __mul24(yg >> 1, pr) + (yg & 1), o = __mul24(e >> 1, pr) + (e & 1);
            acc[o + 2 * x] += acc[og + 2 * x];
        }
    }
    __syncthreads();
}

// Bound on the count of any cell of row y of plane z: a cell of row y is
// reached only by beads of the P slabs z-P+1 .. z and the P row bins
// y-P+1 .. y.  The P row bins of one slab are consecutive (modulo the row
// wrap), so each slab's share is a difference of two bin starts.  Returns
// the largest such bead count over the rows this thread visits.
template <int P>
__device__ __forceinline__ uint32_t stencil_count_max(const uint32_t* __restrict__ bin_start, const Dims d, int z,
                                                      int K, int tid, int nthr) {
    uint32_t mine = 0;
    for (int y = tid; y < d.my; y += nthr) {
        uint32_t lo[P], hi[P], lo2[P], hi2[P];
        const int y0 = y - (P - 1);  // rows y0 .. y, wrapped
#pragma unroll
        for (int c = 0; c < P; ++c) {
            int s = z - c;
            if (s < 0) s += d.mz;
            const int b0 = (K * d.mz + s) * d.my;
            if (y0 >= 0) {
                lo[c] = bin_start[b0 + y0];
                hi[c] = bin_start[b0 + y + 1];
                lo2[c] = hi2[c] = 0u;
            } else {
                lo[c] = bin_start[b0];
                hi[c] = bin_start[b0 + y + 1];
                lo2[c] = bin_start[b0 + d.my + y0];
                hi2[c] = bin_start[b0 + d.my];
            }
        }
        uint32_t sum = 0;
#pragma unroll
        for (int c = 0; c < P; ++c) sum += (hi[c] - lo[c]) + (hi2[c] - lo2[c]);
        mine = mine > sum ? mine : sum;
    }
    return mine;
}

// Scale of the fixed-point spread of a plane: the largest 2^k for which no
// cell can overflow the accumulator, each bead contributing at most wmax to a
// cell whose count of reaching beads is at most maxcount.  Single precision:
// int32 cells, k <= 24; double precision: int64 cells (below 2^62), k <= 50.
template <typename T>
__device__ __forceinline__ T spread_scale(uint32_t maxcount, double wmax, uint32_t* __restrict__ flag, int tid) {
    constexpr int kMax = sizeof(T) == 4 ? 24 : 50, kMin = 8;
    const double limit = sizeof(T) == 4 ? 2147483647.0 : 4611686018427387904.0;
    const double bound = (double)maxcount * wmax + 1.0;
    int k = kMax;
    while (k > kMin && bound * ldexp(1.0, k) >= limit) --k;
    if (bound * ldexp(1.0, k) >= limit && tid == 0) atomicOr(flag, 4u);
    return (T)ldexp(1.0, k);
}

// Scale 2^k of the weighted counts of a plane: every cell's |sum q_j W_j(g)|
// is at most qmax (maxcount wmax + 1), kept below half the integer range
// (the rounding of each contribution adds at most half a unit per bead).
template <typename T>
__device__ __forceinline__ T weighted_scale(uint32_t maxcount, double wmax, double qmax) {
    const double limit = sizeof(T) == 4 ? 2147483647.0 : 4611686018427387904.0;
    const double bound = ((double)maxcount * wmax + 1.0) * qmax;
    if (!(bound > 0.0)) return (T)1;  // no weight on this plane
    int e = 0;
    (void)frexp(limit / bound, &e);  // limit / bound >= 2^(e-1)
    e = e - 2 < -120 ? -120 : (e - 2 > 120 ? 120 : e - 2);
    return (T)ldexp(1.0, e);
}

// Plane z of species K: counts minus their mean N_K/M, then the forward
// transform to the half spectrum H[ky][kx], kx = 0 .. mx/2.  Rows 2p and 2p+1
// are transformed together as one complex row c_2p + i c_2p+1, stored at
// complex offset p * zp, and separated in place, by the lanes that
// transformed them, with the symmetry Z(-k)*: H row 2p lands at p * zp and
// row 2p+1 at p * zp + hxp, i.e. H has row pitch hxp.
// At least four waves per SIMD (128 VGPRs): two 512-thread or one
// 1024-thread workgroup per CU, as the plane's LDS allows.
//
// BATCH: one launch for all members of a batch; the unit map names each
// workgroup's member and plane, and the member's descriptor replaces the
// per-context arguments.
//
// DIR: the directional counts sum_j grad W_j . v_j (vdir) instead of the
// counts, with no mean to subtract and no noise; WSP (with DIR): the weighted
// counts sum_j q_j W_j (spread_plane_weighted).  Both accumulate in fixed
// point at a scale from the plane's count bound and largest bead weight.
//
// COUNTS: write the counts c_K(z) themselves (real, [2][mz][my][mx], x
// fastest) to cout and stop before the transforms.
//
// WSP (with DIR): the weighted counts sum_j q_j W_j, q_j = vdir[4 j + comp],
// instead of the directional ones.
template <typename T, int BLOCK, int P, bool BATCH = false, bool DIR = false, bool COUNTS = false, bool WSP = false>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))
    k_spread_xy(const uint4* __restrict__ pos, const uint32_t* __restrict__ bin_start, const uint32_t* __restrict__ qs,
                cplx<T>* __restrict__ spec, Dims d, FftPlan px, FftPlan py, const cplx<T>* __restrict__ tw, Phys ph,
                uint32_t* __restrict__ flag, const RepDesc* __restrict__ reps, const uint32_t* __restrict__ umap,
                int parity,
                const T* __restrict__ vdir, T* __restrict__ cout, int comp) {
    static_assert(!WSP || DIR, "weighted counts use the floating-point accumulation of DIR");
    using C = cplx<T>;
    using A = typename std::conditional<sizeof(T) == 4, uint32_t, unsigned long long>::type;
    using SA = typename std::conditional<sizeof(T) == 4, int32_t, long long>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ uint32_t smax[BLOCK / 64];
    __shared__ T sqmax[DIR ? BLOCK / 64 : 1];
    C* S = reinterpret_cast<C*>(smem);
    const int tid = threadIdx.x;
    // one XCD takes a run of consecutive planes, whose bead slabs overlap
    int t;
    if constexpr (BATCH) {
        const uint32_t e = umap[xcd_contiguous(blockIdx.x, gridDim.x)];
        const RepDesc& R = reps[e >> 16];
        pos = sizeof(T) == 4 ? R.S.grec : R.S.pos;
        bin_start = R.S.bin_start;
        qs = parity ? R.S.qshift_next : R.S.qshift;
        spec = (C*)R.S.spec;
        d = R.d;
        px = R.px;
        py = R.py;
        tw = (const C*)R.S.tw;
        ph = R.ph;
        flag = R.S.flag;
        t = (int)(e & 0xffffu);
    } else {
        t = xcd_contiguous(blockIdx.x + d.mz * blockIdx.y, 2 * d.mz);
    }
    const int z = t % d.mz, K = t / d.mz;
    const int mx = d.mx, my = d.my, hx = d.hx, hxp = d.hxp, np = d.npair, zp = 2 * hxp;
    const T mean = DIR ? (T)0 : (T)(K ? ph.mean_b : ph.mean_a);
    // Prologue: issue the global loads (twiddles, bin starts) before zeroing
    // the plane, then one barrier.
    C* twl = S + d.npg * zp;
    const int ntw = d.ntw();
    C twv[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) twv[u] = tid + u * BLOCK < ntw ? tw[tid + u * BLOCK] : C{0, 0};
    uint32_t mine = 0;
    T qmine = 0;
    mine = stencil_count_max<P>(bin_start, d, z, K, tid, BLOCK);
    if constexpr (WSP) qmine = weight_max<T, P>(bin_start, d, z, K, vdir, comp, tid, BLOCK);
    else if constexpr (DIR) qmine = dir_weight_max<T, P>(bin_start, d, z, K, vdir, tid, BLOCK);
    for (int i = tid; i < d.npg * zp; i += BLOCK) S[i] = C{0, 0};  // zero bits: integer or float zero
#pragma unroll
    for (int u = 0; u < 3; ++u)
        if (tid + u * BLOCK < ntw) twl[tid + u * BLOCK] = twv[u];
    for (int i = tid + 3 * BLOCK; i < ntw; i += BLOCK) twl[i] = tw[i];
    {
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const uint32_t other = __shfl_xor(mine, o, 64);
            mine = mine > other ? mine : other;
            if constexpr (DIR) {
                const T qo = __shfl_xor(qmine, o, 64);
                qmine = qmine > qo ? qmine : qo;
            }
        }
        if ((tid & 63) == 0) {
            smax[tid >> 6] = mine;
            if constexpr (DIR) sqmax[tid >> 6] = qmine;
        }
    }
    __syncthreads();
    T scale = (T)1;
    {
        uint32_t m = 0;
        T qm = 0;
#pragma unroll
        for (int w = 0; w < BLOCK / 64; ++w) {
            m = m > smax[w] ? m : smax[w];
            if constexpr (DIR) qm = qm > sqmax[w] ? qm : sqmax[w];
        }
        // weighted counts: weight peak wmax; directional: the bound is per bead
        if constexpr (WSP) scale = weighted_scale<T>(m, ph.wmax, (double)qm);
        else if constexpr (DIR) scale = weighted_scale<T>(m, 1.0, (double)qm);
        else scale = spread_scale<T>(m, ph.wmax, flag, tid);
    }
    if constexpr (WSP) {
        spread_plane_weighted<T, P>(reinterpret_cast<A*>(smem), pos, bin_start, qs, d, z, K, vdir, comp, scale, tid,
                                    BLOCK);
        __syncthreads();
        fold_ghosts<A, P>(reinterpret_cast<A*>(smem), d, tid, BLOCK);
    } else if constexpr (DIR) {
        spread_plane_dir<T, P>(reinterpret_cast<A*>(smem), pos, bin_start, qs, d, z, K, vdir, scale, tid, BLOCK);
        __syncthreads();
        fold_ghosts<A, P>(reinterpret_cast<A*>(smem), d, tid, BLOCK);
    } else {
        spread_plane<T, P>(smem, pos, bin_start, qs, d, z, K, scale, tid, BLOCK);
        __syncthreads();
        fold_ghosts<A, P>(reinterpret_cast<A*>(smem), d, tid, BLOCK);
    }
    if constexpr (COUNTS) {
        const T inv = (T)1 / scale;
        const A* Si = reinterpret_cast<const A*>(smem);
        T* dst = cout + ((long long)K * d.mz + z) * (long long)my * mx;
        for (int i = tid; i < my * mx; i += BLOCK) {
            const int y = i / mx, x = i - y * mx;
            dst[i] = (T)(SA)Si[__mul24(y >> 1, 4 * hxp) + (y & 1) + 2 * x] * inv;
        }
        return;
    }
    {
        // counts (minus their mean) of the real cells; zero elsewhere
        const T inv = (T)1 / scale;
        Walk2 w(tid, zp, BLOCK);
        for (int i = tid; i < np * zp; i += BLOCK, w.next()) {
            T vr = 0, vi = 0;
            {
                const A* Si = reinterpret_cast<const A*>(smem);
                const A re = Si[2 * i], im = Si[2 * i + 1];
                if (w.x < mx) {
                    vr = (T)(SA)re * inv - mean;
                    if (2 * w.p + 1 < my) vi = (T)(SA)im * inv - mean;
                }
            }
            S[i] = C{vr, vi};
        }
    }
    __syncthreads();
    {
        const int G = px.group, lane = tid % G;
        for (int p = tid / G; p < np; p += BLOCK / G) {
            const int base = p * zp;
            fft_line<C, 0, false, true>(S, base, 1, px, twl, lane);
            C ra[kPairItems], rb[kPairItems];
#pragma unroll
            for (int u = 0; u < kPairItems; ++u) {
                const int kx = lane + u * G;
                if (kx < hx) {
                    const C a = S[base + kx];
                    const C b = S[base + (kx == 0 ? 0 : mx - kx)];
                    ra[u] = C{(T)0.5 * (a.x + b.x), (T)0.5 * (a.y - b.y)};
                    rb[u] = C{(T)0.5 * (a.y + b.y), (T)0.5 * (b.x - a.x)};
                }
            }
            wave_sync();
#pragma unroll
            for (int u = 0; u < kPairItems; ++u) {
                const int kx = lane + u * G;
                if (kx < hx) {
                    S[hidx(d, 2 * p, kx)] = ra[u];
                    if (2 * p + 1 < my) S[hidx(d, 2 * p + 1, kx)] = rb[u];
                }
            }
            wave_sync();
        }
    }
    __syncthreads();
    // For even mx the columns kx = 0 and kx = mx/2 are real for every row (x
    // transforms of real rows at frequencies 0 and pi).  They share one y
    // transform as Z = H_0 + i H_N, separated afterwards with the symmetry of
    // transforms of real sequences, which saves one of hx lines.
    const bool pair_n = (mx & 1) == 0 && hx > 1;
    if (pair_n) {
        for (int y = tid; y < my; y += BLOCK) S[hidx(d, y, 0)] = C{S[hidx(d, y, 0)].x, S[hidx(d, y, hx - 1)].x};
        __syncthreads();
    }
    if (d.swc) fft_lines<C, 0, true, true>(S, LineMap{d.ylines, d.ylines, 1, 0, hxp, 15}, py, twl, tid, BLOCK);
    else fft_lines<C, 0, false, true>(S, LineMap{d.ylines, d.ylines, 1, 0, hxp, 0}, py, twl, tid, BLOCK);
    __syncthreads();
    if (pair_n) {
        for (int ky = tid; ky <= my / 2; ky += BLOCK) {
            const int kn = ky == 0 ? 0 : my - ky;
            const C zp = S[hidx(d, ky, 0)], zm = S[hidx(d, kn, 0)];
            const C h0 = C{(T)0.5 * (zp.x + zm.x), (T)0.5 * (zp.y - zm.y)};  // (Z(k) + Z(-k)*) / 2
            const C hn = C{(T)0.5 * (zp.y + zm.y), (T)0.5 * (zm.x - zp.x)};  // (Z(k) - Z(-k)*) / 2i
            S[hidx(d, ky, 0)] = h0;
            S[hidx(d, ky, hx - 1)] = hn;
            if (kn != ky) {
                S[hidx(d, kn, 0)] = C{h0.x, -h0.y};
                S[hidx(d, kn, hx - 1)] = C{hn.x, -hn.y};
            }
        }
        __syncthreads();
    }
    C* dst = spec + ((long long)K * d.mz + z) * d.hplane;
    Walk2 w(tid, hx, BLOCK);
    for (int i = tid; i < my * hx; i += BLOCK, w.next()) dst[i] = S[hidx(d, w.p, w.x)];
}

// Contribution of gradient plane z (component a, species K, held in LDS in the
// extended row-pair layout) to the non-bonded force of every bead whose
// stencil reaches the plane: the beads of the P slabs z-P+1 .. z.  A bead of
// slab z - c gets
//   fpart[a][c][j] = -w_z[c] sum_{b,a'} w_y[b] w_x[a'] d_a phi(g0y + b, g0x + a'),
// so that its force component a is the sum of fpart[a][0 .. P-1][j].
template <typename T, int P>
__device__ __forceinline__ void push_plane(const T* __restrict__ Sr, const uint4* __restrict__ pos,
                                           const uint32_t* __restrict__ bin_start, const uint32_t* __restrict__ qs,
                                           const Dims d, int z, int K, int a, long long n, T* __restrict__ fpart,
                                           int tid, int nthr) {
    const uint32_t sx = qs[0], sy = qs[1], sz = qs[2];
    const int pr = 4 * d.hxp;
#pragma unroll
    for (int c = 0; c < P; ++c) {
        int s = z - c;
        if (s < 0) s += d.mz;
        const int b0 = (K * d.mz + s) * d.my;
        const uint32_t j0 = bin_start[b0], j1 = bin_start[b0 + d.my];
        T* out = fpart + ((long long)a * P + c) * n;
        // one bead per thread at a time, the next bead's record loaded while
        // this one is interpolated (beads loaded in a batch with branches
        // between them had each load sunk into its bead's branch and waited
        // on there)
        const uint32_t jt = j0 + (uint32_t)tid;
        if (jt < j1) {
            uint4 qn = pos[jt];
            for (uint32_t j = jt; j < j1; j += (uint32_t)nthr) {
                const uint4 q = qn;
                const uint32_t jn = j + (uint32_t)nthr;
                qn = pos[jn < j1 ? jn : j1 - 1u];
                const BeadFrac<T> bf = bead_frac<T, P>(q, sx, sy, sz, d.mx, d.my, d.mz);
                const int gx = bf.gx;
                T wx[P], wy[P];
                spline_weights<T, P>(bf.fx, wx);
                spline_weights<T, P>(bf.fy, wy);
                T wzs[P];  // only wzs[c] survives unrolling
                spline_weights<T, P>(bf.fz, wzs);
                const T wz = wzs[c];
                const RowOffsets<P> ro(bf.gy, pr);
                T acc = 0;
#pragma unroll
                for (int b = 0; b < P; ++b) {
                    const T* row = Sr + ro.o[b] + 2 * gx;
                    T ra = 0;
#pragma unroll
                    for (int a2 = 0; a2 < P; ++a2) ra += wx[a2] * row[2 * a2];
                    acc += wy[b] * ra;
                }
                out[j] = -wz * acc;
            }
        }
    }
}

// Exact-gradient route (the mesh energy's derivative): the potential plane
// phi_K(z) in LDS gives every bead of the P slabs z-P+1 .. z all three
// components of its plane-c term,
//   fpart[a][c][j] = -sum_{b,a'} d/dx_a [w_x[a'] w_y[b] w_z[c]] phi_K(g0y + b, g0x + a'),
// with dw/dx = (dw/df) / h.  Returns this thread's sum of the values it wrote,
// per axis, in 32.32 fixed point (the mean force enters the centre-of-mass shift).
template <typename T, int P>
__device__ __forceinline__ void push_plane_ad(const T* __restrict__ Sr, const uint4* __restrict__ pos,
                                              const uint32_t* __restrict__ bin_start,
                                              const uint32_t* __restrict__ qs, const Dims d, int z, int K,
                                              long long n, T* __restrict__ fpart, long long fsum[3], int tid,
                                              int nthr) {
    const uint32_t sx = qs[0], sy = qs[1], sz = qs[2];
    const int pr = 4 * d.hxp;
    const T ihx = (T)(d.mx / d.lx), ihy = (T)(d.my / d.ly), ihz = (T)(d.mz / d.lz);
#pragma unroll
    for (int c = 0; c < P; ++c) {
        int s = z - c;
        if (s < 0) s += d.mz;
        const int b0 = (K * d.mz + s) * d.my;
        const uint32_t j0 = bin_start[b0], j1 = bin_start[b0 + d.my];
        // one bead per thread at a time, the next bead's record prefetched
        // (see push_plane)
        const uint32_t jt = j0 + (uint32_t)tid;
        if (jt < j1) {
            uint4 qn = pos[jt];
            for (uint32_t j = jt; j < j1; j += (uint32_t)nthr) {
                const uint4 q = qn;
                const uint32_t jn = j + (uint32_t)nthr;
                qn = pos[jn < j1 ? jn : j1 - 1u];
                const BeadFrac<T> bf = bead_frac<T, P>(q, sx, sy, sz, d.mx, d.my, d.mz);
                const int gx = bf.gx;
                T wx[P], wy[P], dwx[P], dwy[P];
                spline_weights<T, P>(bf.fx, wx);
                spline_weights<T, P>(bf.fy, wy);
                spline_dweights<T, P>(bf.fx, dwx);
                spline_dweights<T, P>(bf.fy, dwy);
                const T fz = bf.fz;
                T wzs[P], dwzs[P];  // only entry c survives unrolling
                spline_weights<T, P>(fz, wzs);
                spline_dweights<T, P>(fz, dwzs);
                const RowOffsets<P> ro(bf.gy, pr);
                T ax = 0, ay = 0, az = 0;
#pragma unroll
                for (int b = 0; b < P; ++b) {
                    const T* row = Sr + ro.o[b] + 2 * gx;
                    T r = 0, rx = 0;
#pragma unroll
                    for (int a2 = 0; a2 < P; ++a2) {
                        const T v = row[2 * a2];
                        r += wx[a2] * v;
                        rx += dwx[a2] * v;
                    }
                    ax += wy[b] * rx;
                    ay += dwy[b] * r;
                    az += wy[b] * r;
                }
                const T f[3] = {-ihx * wzs[c] * ax, -ihy * wzs[c] * ay, -ihz * dwzs[c] * az};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    fpart[((long long)a * P + c) * n + j] = f[a];
                    fsum[a] += llrint((double)f[a] * kTwo32);
                }
            }
        }
    }
}

// Local part of the ik-route force Jacobian, transposed: with the gradient
// plane d_a phi_K(z) in LDS, every bead j of the P slabs z-P+1 .. z gets its
// plane-c term of
//   vdir[4 j + a] sum_g d_b W_j(g) d_a phi_K(g),   b = x, y, z,
// written to fpart[b][c][j].
template <typename T, int P>
__device__ __forceinline__ void push_plane_local(const T* __restrict__ Sr, const uint4* __restrict__ pos,
                                                 const uint32_t* __restrict__ bin_start,
                                                 const uint32_t* __restrict__ qs, const Dims d, int z, int K, int a,
                                                 long long n, const T* __restrict__ vdir, T* __restrict__ fpart,
                                                 int tid, int nthr) {
    const uint32_t sx = qs[0], sy = qs[1], sz = qs[2];
    const int pr = 4 * d.hxp;
    const T ihx = (T)(d.mx / d.lx), ihy = (T)(d.my / d.ly), ihz = (T)(d.mz / d.lz);
#pragma unroll
    for (int c = 0; c < P; ++c) {
        int s = z - c;
        if (s < 0) s += d.mz;
        const int b0 = (K * d.mz + s) * d.my;
        const uint32_t j0 = bin_start[b0], j1 = bin_start[b0 + d.my];
        for (uint32_t j = j0 + (uint32_t)tid; j < j1; j += (uint32_t)nthr) {
            const uint4 q = pos[j];
            const T lam = vdir[4 * (long long)j + a];
            const BeadFrac<T> bf = bead_frac<T, P>(q, sx, sy, sz, d.mx, d.my, d.mz);
            const int gx = bf.gx;
            T wx[P], wy[P], dwx[P], dwy[P], wzs[P], dwzs[P];  // only entry c of the z weights survives
            spline_weights<T, P>(bf.fx, wx);
            spline_weights<T, P>(bf.fy, wy);
            spline_dweights<T, P>(bf.fx, dwx);
            spline_dweights<T, P>(bf.fy, dwy);
            spline_weights<T, P>(bf.fz, wzs);
            spline_dweights<T, P>(bf.fz, dwzs);
            const RowOffsets<P> ro(bf.gy, pr);
            T ax = 0, ay = 0, az = 0;
#pragma unroll
            for (int b = 0; b < P; ++b) {
                const T* row = Sr + ro.o[b] + 2 * gx;
                T r = 0, rx = 0;
#pragma unroll
                for (int a2 = 0; a2 < P; ++a2) {
                    const T v = row[2 * a2];
                    r += wx[a2] * v;
                    rx += dwx[a2] * v;
                }
                ax += wy[b] * rx;
                ay += dwy[b] * r;
                az += wy[b] * r;
            }
            fpart[((long long)0 * P + c) * n + j] = lam * ihx * wzs[c] * ax;
            fpart[((long long)1 * P + c) * n + j] = lam * ihy * wzs[c] * ay;
            fpart[((long long)2 * P + c) * n + j] = lam * ihz * dwzs[c] * az;
        }
    }
}

// Hessian-vector products: with the potential plane phi_K(z) in LDS, every
// bead j of the P slabs z-P+1 .. z gets its plane-c term of
//   (H v)_a = sum_b sum_g d^2 W_j(g) / dx_a dx_b v_jb phi_K(g),
// written (with a plus sign) to fpart[a][c][j]; the weights' second
// derivatives come from the same compile-time spline pieces (P >= 3).
template <typename T, int P>
__device__ __forceinline__ void push_plane_hess(const T* __restrict__ Sr, const uint4* __restrict__ pos,
                                                const uint32_t* __restrict__ bin_start,
                                                const uint32_t* __restrict__ qs, const Dims d, int z, int K,
                                                long long n, const T* __restrict__ vdir, T* __restrict__ fpart,
                                                int tid, int nthr) {
    const uint32_t sx = qs[0], sy = qs[1], sz = qs[2];
    const int pr = 4 * d.hxp;
    const T ihx = (T)(d.mx / d.lx), ihy = (T)(d.my / d.ly), ihz = (T)(d.mz / d.lz);
#pragma unroll
    for (int c = 0; c < P; ++c) {
        int s = z - c;
        if (s < 0) s += d.mz;
        const int b0 = (K * d.mz + s) * d.my;
        const uint32_t j0 = bin_start[b0], j1 = bin_start[b0 + d.my];
        for (uint32_t j = j0 + (uint32_t)tid; j < j1; j += (uint32_t)nthr) {
            const uint4 q = pos[j];
            const BeadFrac<T> bf = bead_frac<T, P>(q, sx, sy, sz, d.mx, d.my, d.mz);
            const int gx = bf.gx, gy = bf.gy;
            T wx[P], wy[P], dwx[P], dwy[P], ddx[P], ddy[P];
            const T fx = bf.fx, fy = bf.fy;
            spline_weights<T, P>(fx, wx);
            spline_weights<T, P>(fy, wy);
            spline_dweights<T, P>(fx, dwx);
            spline_dweights<T, P>(fy, dwy);
            spline_d2weights<T, P>(fx, ddx);
            spline_d2weights<T, P>(fy, ddy);
            const T fz = bf.fz;
            T wzs[P], dwzs[P], ddzs[P];  // only entry c survives unrolling
            spline_weights<T, P>(fz, wzs);
            spline_dweights<T, P>(fz, dwzs);
            spline_d2weights<T, P>(fz, ddzs);
            const RowOffsets<P> ro(gy, pr);
            // node sums of phi against products of 1-D factors: s_ab = sum w^(a)_x w^(b)_y phi
            T s00 = 0, s10 = 0, s01 = 0, s20 = 0, s11 = 0, s02 = 0;
#pragma unroll
            for (int b = 0; b < P; ++b) {
                const T* row = Sr + ro.o[b] + 2 * gx;
                T r0 = 0, r1 = 0, r2 = 0;
#pragma unroll
                for (int a2 = 0; a2 < P; ++a2) {
                    const T v = row[2 * a2];
                    r0 += wx[a2] * v;
                    r1 += dwx[a2] * v;
                    r2 += ddx[a2] * v;
                }
                s00 += wy[b] * r0;
                s10 += wy[b] * r1;
                s01 += dwy[b] * r0;
                s20 += wy[b] * r2;
                s11 += dwy[b] * r1;
                s02 += ddy[b] * r0;
            }
            const T wz = wzs[c], dwz = dwzs[c], ddz = ddzs[c];
            const T hxx = ihx * ihx * wz * s20, hyy = ihy * ihy * wz * s02, hzz = ihz * ihz * ddz * s00;
            const T hxy = ihx * ihy * wz * s11, hxz = ihx * ihz * dwz * s10, hyz = ihy * ihz * dwz * s01;
            const T vx = vdir[4 * (long long)j], vy = vdir[4 * (long long)j + 1], vz = vdir[4 * (long long)j + 2];
            fpart[((long long)0 * P + c) * n + j] = hxx * vx + hxy * vy + hxz * vz;
            fpart[((long long)1 * P + c) * n + j] = hxy * vx + hyy * vy + hyz * vz;
            fpart[((long long)2 * P + c) * n + j] = hxz * vx + hyz * vy + hzz * vz;
        }
    }
}

// Inverse transform of one plane held in LDS as a half spectrum (row pitch
// hxp, swizzled as hidx): inverse FFT along y, then complex-to-real along x
// with rows 2p and 2p+1 carried as the real and imaginary parts of one
// complex row, packed in place at complex offset p * zp by the lanes that
// then transform it.  Called by nthr threads (tid < nthr) after a barrier;
// every thread of the block takes part in its barriers, so two halves of a
// block may transform two planes side by side.  Ends without a barrier.
template <typename T>
__device__ __forceinline__ void inverse_xy_transform(cplx<T>* __restrict__ S, const Dims d, const FftPlan px,
                                                     const FftPlan py, const cplx<T>* __restrict__ twl, int tid,
                                                     int nthr) {
    using C = cplx<T>;
    const int mx = d.mx, my = d.my, hx = d.hx, hxp = d.hxp, np = d.npair, zp = 2 * hxp;
    // For even mx the columns kx = 0 and kx = mx/2 transform back to real
    // rows; one y transform of Z = G_0 + i G_N gives both.
    const bool pair_n = (mx & 1) == 0 && hx > 1;
    if (pair_n) {
        for (int y = tid; y < my; y += nthr) {
            const C g0 = S[hidx(d, y, 0)], gn = S[hidx(d, y, hx - 1)];
            S[hidx(d, y, 0)] = C{g0.x - gn.y, g0.y + gn.x};
        }
        __syncthreads();
    }
    if (d.swc) fft_lines<C, 1, true, true>(S, LineMap{d.ylines, d.ylines, 1, 0, hxp, 15}, py, twl, tid, nthr);
    else fft_lines<C, 1, false, true>(S, LineMap{d.ylines, d.ylines, 1, 0, hxp, 0}, py, twl, tid, nthr);
    __syncthreads();
    if (pair_n) {
        for (int y = tid; y < my; y += nthr) {
            const C zv = S[hidx(d, y, 0)];
            S[hidx(d, y, 0)] = C{zv.x, (T)0};
            S[hidx(d, y, hx - 1)] = C{zv.y, (T)0};
        }
        __syncthreads();
    }
    {
        const int G = px.group, lane = tid % G;
        for (int p = tid / G; p < np; p += nthr / G) {
            const int base = p * zp;
            const bool odd = 2 * p + 1 < my;
            C rz[kPairItems];
#pragma unroll
            for (int u = 0; u < kPairItems; ++u) {
                const int x = lane + u * G;
                if (x < mx) {
                    C A, B;
                    if (x < hx) {
                        A = S[hidx(d, 2 * p, x)];
                        B = odd ? S[hidx(d, 2 * p + 1, x)] : C{0, 0};
                    } else {
                        const int xs = mx - x;
                        const C a0 = S[hidx(d, 2 * p, xs)];
                        const C b0 = odd ? S[hidx(d, 2 * p + 1, xs)] : C{0, 0};
                        A = C{a0.x, -a0.y};
                        B = C{b0.x, -b0.y};
                    }
                    rz[u] = C{A.x - B.y, A.y + B.x};
                }
            }
            wave_sync();
#pragma unroll
            for (int u = 0; u < kPairItems; ++u) {
                const int x = lane + u * G;
                if (x < mx) S[base + x] = rz[u];
            }
            wave_sync();
            fft_line<C, 1, false, true>(S, base, 1, px, twl, lane);
        }
    }
}

// Fill the ghost columns and rows of a real plane in the extended row-pair
// layout (ghost columns of the real rows, then ghost rows, ghost columns
// included).  Starts after a barrier and ends with one.
template <typename T, int P>
__device__ __forceinline__ void fill_ghosts(T* __restrict__ Sr, const Dims d, int tid, int nthr) {
    if constexpr (P > 1) {
        const int pr = 4 * d.hxp, mx = d.mx, my = d.my;
        for (int i = tid; i < my * (P - 1); i += nthr) {
            const int y = i / (P - 1), e = i - y * (P - 1);
            const int o = __mul24(y >> 1, pr) + (y & 1);
            Sr[o + 2 * (mx + e)] = Sr[o + 2 * e];
        }
        __syncthreads();
        for (int i = tid; i < (P - 1) * (mx + P - 1); i += nthr) {
            const int e = i / (mx + P - 1), x = i - e * (mx + P - 1);
            const int yg = my + e;
            Sr[__mul24(yg >> 1, pr) + (yg & 1) + 2 * x] = Sr[__mul24(e >> 1, pr) + (e & 1) + 2 * x];
        }
    }
    __syncthreads();
}

// Inverse (one workgroup per plane z, species K and axis a = x, y, z): build
// the half spectrum of d_a phi_K on plane z (row pitch hxp), inverse FFT
// along y, then complex-to-real along x with rows 2p and 2p+1 carried as the
// real and imaginary parts of one complex row, packed in place at complex
// offset p * zp by the lanes that then transform it; the ghost columns and
// rows are filled in, and the finished plane d_a phi_K(z) is interpolated
// onto the beads that reach it.
//
// AD: exact-gradient route instead: one workgroup per plane z and species K
// transforms phi_K itself and interpolates all three components with the
// weight derivatives (push_plane_ad); fsum_part receives the workgroup's
// force sums (32.32 fixed point).
//
// BATCH (ik route only): one launch for all members of a batch, as for the
// spread.
//
// HESS (with AD): the potential plane's Hessian-vector terms (push_plane_hess,
// vdir) instead of the force terms.
//
// FIELD (with AD): interpolate a given real field psi_K ([2][mz][my][mx],
// x fastest) instead of transforming a spectrum: the forces
// -sum_g grad W_i(g) psi_{s_i}(g).
//
// XM (ik route, one component a = comp, one workgroup per plane and
// species): 1 -- the local part of the transposed force Jacobian against
// vdir (push_plane_local); 2 -- store the gradient plane d_a phi_K(z) in
// fout ([2][mz][my][mx], x fastest), adding to what is there when comp > 0.
//
// The ik route's stepping pass (XM = 0, not batched) runs on a 1-D grid over
// units t0 .. t0 + gridDim.x - 1 of the 6 mz units t = (K mz + z) 3 + a.
template <typename T, int BLOCK, int P, bool AD, bool BATCH = false, bool HESS = false, bool FIELD = false,
          int XM = 0>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 2)))
    k_xy_c2r(const cplx<T>* __restrict__ zout, T* __restrict__ fpart, Dims d, FftPlan px, FftPlan py,
             const cplx<T>* __restrict__ tw, Phys ph, const uint4* __restrict__ pos,
             const uint32_t* __restrict__ bin_start, const uint32_t* __restrict__ qs, long long n,
             long long* __restrict__ fsum_part, const RepDesc* __restrict__ reps, const uint32_t* __restrict__ umap,
             int parity, const T* __restrict__ vdir, const T* __restrict__ field, int comp, T* __restrict__ fout,
             int t0) {
    static_assert(XM == 0 || (!AD && !BATCH), "the Jacobian modes run on the ik route of one context");
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    C* S = reinterpret_cast<C*>(smem);
    const int tid = threadIdx.x;
    // one XCD takes the three axes of a run of consecutive planes of one
    // species: all of them read the same bead slabs
    int t;
    if constexpr (BATCH) {
        static_assert(!AD, "batched steps use the ik route");
        const uint32_t e = umap[xcd_contiguous(blockIdx.x, gridDim.x)];
        const RepDesc& R = reps[e >> 16];
        zout = (const C*)R.S.zout;
        fpart = (T*)R.S.fpart;
        d = R.d;
        px = R.px;
        py = R.py;
        tw = (const C*)R.S.tw;
        ph = R.ph;
        pos = sizeof(T) == 4 ? R.S.grec : R.S.pos;
        bin_start = R.S.bin_start;
        qs = parity ? R.S.qshift_next : R.S.qshift;
        n = R.S.n;
        t = (int)(e & 0xffffu);
    } else if constexpr (XM != 0) {
        t = xcd_contiguous(blockIdx.x + d.mz * blockIdx.y, 2 * d.mz);
    } else if constexpr (AD) {
        t = xcd_contiguous(blockIdx.x + d.mz * blockIdx.y, 2 * d.mz);
    } else {
        t = t0 + xcd_contiguous(blockIdx.x, gridDim.x);  // units t0 .. t0 + gridDim.x - 1 of 6 mz
    }
    constexpr bool ONE = AD || XM != 0;  // one workgroup per plane and species
    const int a = AD ? 2 : (XM != 0 ? comp : t % 3);
    const int z = ONE ? t % d.mz : (t / 3) % d.mz, K = ONE ? t / d.mz : t / (3 * d.mz);
    const int mx = d.mx, my = d.my, hx = d.hx, hxp = d.hxp, zp = 2 * hxp;
    const T kfx = (T)(kTwoPi / ph.lx), kfy = (T)(kTwoPi / ph.ly);
    C* twl = S + d.npg * zp;
    const int ntw = d.ntw();
    {
        if constexpr (FIELD) {
            T* Sf = reinterpret_cast<T*>(smem);
            const T* src = field + ((long long)K * d.mz + z) * (long long)my * mx;
            for (int i = tid; i < my * mx; i += BLOCK) {
                const int y = i / mx, x = i - y * mx;
                Sf[__mul24(y >> 1, 4 * hxp) + (y & 1) + 2 * x] = src[i];
            }
        } else {
            C twv[3];  // twiddles, loaded with the plane and stored after it
#pragma unroll
            for (int u = 0; u < 3; ++u) twv[u] = tid + u * BLOCK < ntw ? tw[tid + u * BLOCK] : C{0, 0};
            // the plane's half spectrum, eighteen loads in flight per thread
            const C* src = zout + ((long long)(a < 2 || AD ? K : 2 + K) * d.mz + z) * d.hplane;
            constexpr int LB = 18;
            const int tot = my * hx;
            Walk2 w(tid, hx, BLOCK);
            for (int i0 = tid; i0 < tot; i0 += LB * BLOCK) {
                C v[LB];
#pragma unroll
                for (int u = 0; u < LB; ++u) {
                    const int i = i0 + u * BLOCK;
                    v[u] = i < tot ? src[i] : C{0, 0};
                }
#pragma unroll
                for (int u = 0; u < LB; ++u) {
                    if (i0 + u * BLOCK < tot) {
                        const int ky = w.p, kx = w.x;
                        C vv = v[u];
                        if (a == 0) {
                            const T k = (2 * kx == mx) ? (T)0 : kfx * (T)kx;
                            vv = C{-k * vv.y, k * vv.x};
                        } else if (a == 1) {
                            const int ny = ky > my / 2 ? ky - my : ky;
                            const T k = (2 * ky == my) ? (T)0 : kfy * (T)ny;
                            vv = C{-k * vv.y, k * vv.x};
                        }
                        S[hidx(d, ky, kx)] = vv;
                    }
                    w.next();
                }
            }
#pragma unroll
            for (int u = 0; u < 3; ++u)
                if (tid + u * BLOCK < ntw) twl[tid + u * BLOCK] = twv[u];
            for (int i = tid + 3 * BLOCK; i < ntw; i += BLOCK) twl[i] = tw[i];
            __syncthreads();
            inverse_xy_transform<T>(S, d, px, py, twl, tid, BLOCK);
        }
        __syncthreads();
        T* Sr = reinterpret_cast<T*>(smem);
        if constexpr (XM == 2) {
            // rows 2p and 2p+1 are the real and imaginary parts of complex row p
            T* dst = fout + ((long long)K * d.mz + z) * (long long)my * mx;
            for (int i = tid; i < my * mx; i += BLOCK) {
                const int y = i / mx, x = i - y * mx;
                const T v = Sr[__mul24(y >> 1, 4 * hxp) + (y & 1) + 2 * x];
                dst[i] = comp > 0 ? dst[i] + v : v;
            }
            return;
        }
        fill_ghosts<T, P>(Sr, d, tid, BLOCK);
        if constexpr (AD && HESS) {
            push_plane_hess<T, P>(Sr, pos, bin_start, qs, d, z, K, n, vdir, fpart, tid, BLOCK);
        } else if constexpr (AD) {
            __shared__ long long fred[3 * (BLOCK / 64)];
            long long fsum[3] = {0, 0, 0};
            push_plane_ad<T, P>(Sr, pos, bin_start, qs, d, z, K, n, fpart, fsum, tid, BLOCK);
            block_sum<long long, 3>(fsum, fred, tid, BLOCK);
            if (tid == 0)
                for (int q = 0; q < 3; ++q) fsum_part[(K * d.mz + z) * 3 + q] = fsum[q];
        } else if constexpr (XM == 1) {
            push_plane_local<T, P>(Sr, pos, bin_start, qs, d, z, K, a, n, vdir, fpart, tid, BLOCK);
        } else {
            push_plane<T, P>(Sr, pos, bin_start, qs, d, z, K, a, n, fpart, tid, BLOCK);
        }
    }
}

// ------------------------------------------------------------ z pass + k-space multiply

// Column block c0 .. c0+cb-1 of the flattened (ky, kx) half-spectrum plane,
// all z.  After the forward z FFT the spectra c^_A, c^_B become
//   Phi^_K = (u^/N) sum_L eps_KL c^_L,  eps_AA = eps_BB = kappa, eps_AB = chi + kappa,
// (the k = 0 field has no gradient), and both Phi^_K and ik_z Phi^_K are
// transformed back along z.  The kernel u^ is separable: u^ = t_x(kx) t_y(ky)
// t_z(kz) with per-axis float64 tables utab (exp(-a^2 k^2) factors, or the
// transforms of the node-sampled Gaussian), combined in LDS once per block.
// With `want_energy` the block also accumulates, in float64 over the half
// spectrum (weight 2 for kx strictly between 0 and mx/2):
//   sum u^ Re(c^_A* c^_B), sum_{k!=0} u^ |c^_A + c^_B|^2 and, per axis,
//   sum k_a^2 v^ [(chi/N) Re(c^_A* c^_B) + (kappa/2N) |c^_+|^2],
// v^ = exp(-a^2 k^2) (tables vtab) for the virial.
//
// LDS: [4 mz][cbp] complex with the odd pitch cbp = cb | 1 (the radix-8
// outputs of a line, eight rows apart, then spread over four LDS bank
// groups), twiddles, then the tables (z_lds_bytes).
struct ZColumn {
    double uxy, vxy, kx, ky, w;  // kernel and analytic factors of (kx, ky) (0 past the last column),
                                 // wavenumbers, energy weight
};
struct ZPlane {
    double uz, vz, kz;  // kernel and analytic factors of kz, wavenumber
};

//
// While stepping (noise_part given), the last block, whose column range is
// the shortest, also forms the step's centre-of-mass shift: the forces sum to
// zero exactly (pairwise bonds; the ik route with the Nyquist derivative
// zeroed), so the mean displacement is sqrt(2 kT dt/gamma) times the mean
// Gaussian increment, summed per 256-bead block (k_noise_sum, or the previous
// step's scatter).
// ELEC: the Coulomb kernel of Gaussian-smeared per-species charges joins the
// pair kernel: Phi^_K += q_K W_e rho^_e with W_e = (4 pi l_B / V)
// exp(-a_e^2 k^2) / k^2 and rho^_e = q_A c^_A + q_B c^_B (k = 0 left out),
// and the energy partials gain sum W_e |rho^_e|^2 and its virial terms.
// BATCH: one launch for all members of a batch (stepping only: noise sums
// given, four outputs); each member's last column block forms its shift.
// This thread's share of the sums over blocks of part[3 blk + a], a < 3, nb
// blocks (nb > 0): eight blocks' words in flight per thread (the last loads
// clamped to block nb - 1 and discarded).
template <int NTHR>
__device__ __forceinline__ void noise_total(const long long* __restrict__ part, long long nb, long long v[3]) {
    constexpr int U = 8;
    for (long long i0 = threadIdx.x; i0 < nb; i0 += U * NTHR) {
        long long x[U][3];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long i = i0 + (long long)u * NTHR, ic = i < nb ? i : nb - 1;
#pragma unroll
            for (int a = 0; a < 3; ++a) x[u][a] = part[3 * ic + a];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int a = 0; a < 3; ++a) v[a] += i0 + (long long)u * NTHR < nb ? x[u][a] : 0;
    }
}

template <typename T, int BLOCK, int ENERGY_ONLY, bool ELEC, bool BATCH = false>
__global__ void __launch_bounds__(BLOCK) k_z_kmul(const cplx<T>* __restrict__ spec, cplx<T>* __restrict__ zout, Dims d,
                                                  FftPlan pz, const cplx<T>* __restrict__ tw, Phys ph, int cb,
                                                  double* __restrict__ epart, int want_energy,
                                                  const long long* __restrict__ noise_part, long long n,
                                                  const uint32_t* __restrict__ qs, uint32_t* __restrict__ qs_next,
                                                  const double* __restrict__ utab, const double* __restrict__ vtab,
                                                  int nout, const RepDesc* __restrict__ reps,
                                                  const uint32_t* __restrict__ umap, int parity) {
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[(ELEC ? 9 : 5) * (BLOCK / 64)];
    int blk, nblk;
    if constexpr (BATCH) {
        const uint32_t e = umap[blockIdx.x];
        const RepDesc& R = reps[e >> 16];
        spec = (const C*)R.S.spec;
        zout = (C*)R.S.zout;
        d = R.d;
        pz = R.pz;
        tw = (const C*)R.S.tw;
        ph = R.ph;
        cb = R.z_cols;
        epart = R.S.epart;
        noise_part = R.S.noise_part;
        n = R.S.n;
        qs = parity ? R.S.qshift_next : R.S.qshift;
        qs_next = parity ? R.S.qshift : R.S.qshift_next;
        utab = R.S.utab;
        vtab = R.S.vtab;
        blk = (int)(e & 0xffffu);
        nblk = R.n_zblocks;
    } else {
        // neighbouring column blocks share cache lines at their edges: keep them on one XCD (own L2)
        blk = xcd_contiguous(blockIdx.x, gridDim.x);
        nblk = gridDim.x;
    }
    if (noise_part && blk == nblk - 1) {
        __shared__ long long nred[3 * (BLOCK / 64)];
        long long v[3] = {0, 0, 0};
        const long long nb = (n + 255) / 256;  // the 256-bead blocks that summed the step's noise
        if (nb > 0) noise_total<BLOCK>(noise_part, nb, v);
        block_sum<long long, 3>(v, nred, threadIdx.x, BLOCK);
        if (threadIdx.x == 0) {
            const double L[3] = {ph.lx, ph.ly, ph.lz};
            for (int a = 0; a < 3; ++a) {
                long long shift = 0;
                if (ph.com_correct && n > 0) shift = llround(ph.noise_amp * ((double)v[a] * kInvTwo32) / (double)n * (kTwo32 / L[a]));
                qs_next[a] = qs[a] + (uint32_t)shift;
            }
            qs_next[3] = 0u;
        }
    }
    C* b0 = reinterpret_cast<C*>(smem);
    const int tid = threadIdx.x;
    const int mz = d.mz, my = d.my, mx = d.mx, hx = d.hx;
    const int cbp = cb | 1;
    C* twl = b0 + 4 * mz * cbp;
    const int ntw = d.ntw();
    C twv[2];  // twiddles, loaded with the spectra and stored after them
#pragma unroll
    for (int u = 0; u < 2; ++u) twv[u] = tid + u * BLOCK < ntw ? tw[tid + u * BLOCK] : C{0, 0};
    ZPlane* zt = reinterpret_cast<ZPlane*>(b0 + 4 * mz * cbp + ntw);
    ZColumn* ct = reinterpret_cast<ZColumn*>(zt + mz);
    const int cn = (int)d.hplane;
    const int c0 = blk * cb;
    const double kfx = kTwoPi / ph.lx, kfy = kTwoPi / ph.ly, kfz = kTwoPi / ph.lz;
    {
        // both spectra of the block's columns, nine loads in flight per thread
        constexpr int LB = 9;
        const int tot = 2 * mz * cb;
        Walk2 w(tid, cb, BLOCK);
        for (int i0 = tid; i0 < tot; i0 += LB * BLOCK) {
            C v[LB];
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                const int i = i0 + u * BLOCK;
                v[u] = C{0, 0};
                if (i < tot) {
                    const int row = w.p, j = w.x;
                    if (c0 + j < cn) v[u] = spec[(long long)row * cn + c0 + j];
                }
                w.next();
            }
            Walk2 w2(i0, cb, BLOCK);
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                if (i0 + u * BLOCK < tot) b0[w2.p * cbp + w2.x] = v[u];
                w2.next();
            }
        }
        for (int z = tid; z < mz; z += BLOCK) {
            const double kz = kfz * (double)(z > mz / 2 ? z - mz : z);
            zt[z] = ZPlane{utab[mx + my + z], vtab[mx + my + z], kz};
        }
        for (int j = tid; j < cb; j += BLOCK) {
            const int c = c0 + j;
            const int ky = c / hx, kx = c - ky * hx;
            const double kxv = kfx * (double)kx, kyv = kfy * (double)(ky > my / 2 ? ky - my : ky);
            const bool in = c < cn;
            ct[j] = ZColumn{in ? utab[kx] * utab[mx + ky] : 0.0, in ? vtab[kx] * vtab[mx + ky] : 0.0, kxv, kyv,
                            (kx == 0 || 2 * kx == mx) ? 1.0 : 2.0};
        }
#pragma unroll
        for (int u = 0; u < 2; ++u)
            if (tid + u * BLOCK < ntw) twl[tid + u * BLOCK] = twv[u];
        for (int i = tid + 2 * BLOCK; i < ntw; i += BLOCK) twl[i] = tw[i];
    }
    __syncthreads();
    fft_lines<C, 0>(b0, LineMap{2 * cb, cb, 1, mz * cbp, cbp, 0}, pz, twl, tid, BLOCK);
    __syncthreads();

    constexpr int NACC = ELEC ? 9 : 5;
    double acc[NACC];
#pragma unroll
    for (int q = 0; q < NACC; ++q) acc[q] = 0.0;
    const T inv_n = (T)ph.inv_n, kap = (T)ph.kappa, cpk = (T)(ph.chi + ph.kappa);
    {
        Walk2 w(tid, cb, BLOCK);
        for (int i = tid; i < mz * cb; i += BLOCK, w.next()) {
            const int z = w.p, j = w.x;
            const C A = b0[z * cbp + j], B = b0[(mz + z) * cbp + j];
            const ZColumn col = ct[j];
            const ZPlane pl = zt[z];
            C PA{0, 0}, PB{0, 0}, QA{0, 0}, QB{0, 0};
            if (c0 + j < cn && (c0 + j != 0 || z != 0)) {
                const T f = (T)col.uxy * (T)pl.uz * inv_n;
                PA = C{f * (kap * A.x + cpk * B.x), f * (kap * A.y + cpk * B.y)};
                PB = C{f * (cpk * A.x + kap * B.x), f * (cpk * A.y + kap * B.y)};
                if constexpr (ELEC) {
                    // k^2 > 0: the k = 0 mode is excluded above
                    const double k2 = col.kx * col.kx + col.ky * col.ky + pl.kz * pl.kz;
                    const double we = ph.lb4v * exp(-ph.ae2 * k2) / k2;
                    const T rx = (T)ph.qa * A.x + (T)ph.qb * B.x, ry = (T)ph.qa * A.y + (T)ph.qb * B.y;
                    const T wa = (T)(we * ph.qa), wb = (T)(we * ph.qb);
                    PA.x += wa * rx;
                    PA.y += wa * ry;
                    PB.x += wb * rx;
                    PB.y += wb * ry;
                    if (want_energy) {
                        const double dx = ph.qa * (double)A.x + ph.qb * (double)B.x;
                        const double dy = ph.qa * (double)A.y + ph.qb * (double)B.y;
                        const double e = col.w * we * (dx * dx + dy * dy);
                        const double t = 1.0 / k2 + ph.ae2;
                        acc[5] += e;
                        acc[6] += e * col.kx * col.kx * t;
                        acc[7] += e * col.ky * col.ky * t;
                        acc[8] += e * pl.kz * pl.kz * t;
                    }
                }
                const T kzd = (2 * z == mz) ? (T)0 : (T)pl.kz;
                QA = C{-kzd * PA.y, kzd * PA.x};
                QB = C{-kzd * PB.y, kzd * PB.x};
                if (want_energy) {
                    const double uh = col.w * col.uxy * pl.uz;
                    const double vh = col.w * col.vxy * pl.vz;
                    const double cross = (double)A.x * B.x + (double)A.y * B.y;
                    const double sx = (double)A.x + B.x, sy = (double)A.y + B.y;
                    const double plus = sx * sx + sy * sy;
                    const double core = vh * (ph.chi * ph.inv_n * cross + 0.5 * ph.kappa * ph.inv_n * plus);
                    acc[0] += uh * cross;
                    acc[1] += uh * plus;
                    acc[2] += col.kx * col.kx * core;
                    acc[3] += col.ky * col.ky * core;
                    acc[4] += pl.kz * pl.kz * core;
                }
            }
            // k = 0 of the mean-subtracted counts is zero; the constant
            // chi N_A N_B / N is added when the partials are reduced.
            if (!ENERGY_ONLY) {
                b0[z * cbp + j] = PA;
                b0[(mz + z) * cbp + j] = PB;
                if (nout == 4) {
                    b0[(2 * mz + z) * cbp + j] = QA;
                    b0[(3 * mz + z) * cbp + j] = QB;
                }
            }
        }
    }
    if (want_energy) {
        block_sum<double, NACC>(acc, red, tid, BLOCK);
        if (tid == 0)
            for (int q = 0; q < kEpart; ++q) epart[blk * kEpart + q] = q < NACC ? acc[q] : 0.0;
    }
    if (ENERGY_ONLY) return;
    __syncthreads();
    fft_lines<C, 1>(b0, LineMap{nout * cb, cb, 1, mz * cbp, cbp, 0}, pz, twl, tid, BLOCK);
    __syncthreads();
    {
        Walk2 w(tid, cb, BLOCK);
        for (int i = tid; i < nout * mz * cb; i += BLOCK, w.next()) {
            const int c = c0 + w.x;
            if (c < cn) zout[(long long)w.p * cn + c] = b0[w.p * cbp + w.x];
        }
    }
}

// ------------------------------------------------------------ gather + bonds + update

// Rank of the calling lane among the active lanes of its wavefront that hold
// the same key in one run of consecutive lanes; the run's first lane takes
// the whole run's places in the bin with a single atomic.
__device__ __forceinline__ uint32_t bin_rank(uint32_t kb, bool active, uint32_t* __restrict__ counts) {
    const int lane = threadIdx.x & 63;
    const uint32_t prev = __shfl_up(kb, 1, 64);
    const bool head = !active || lane == 0 || prev != kb;
    const unsigned long long hm = __ballot(head);
    const unsigned long long upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    const int hl = 63 - __clzll(hm & upto);
    const unsigned long long above = hm & ~upto;
    const int nl = above ? __ffsll((long long)above) - 1 : 64;
    uint32_t base = 0;
    if (active && lane == hl) base = atomicAdd(&counts[kb], (uint32_t)(nl - hl));
    base = __shfl(base, hl, 64);
    return base + (uint32_t)(lane - hl);
}

// Ranks r[b] of a workgroup's beads in their bins (keys kb[b], active act[b]).
// The beads of a workgroup are consecutive in the sorted order and move at
// most a few rows or planes per step, so their new keys fall in a narrow
// range: the workgroup counts its beads per key in LDS over a window of
// kRankWin keys from its smallest key, then reserves each key's places with a
// single global atomic; a bead whose key lies beyond the window takes an
// atomic of its own.  Called by all BLOCK threads.
constexpr int kRankWin = 1024;
template <int NB, int BLOCK>
__device__ __forceinline__ void block_rank(const uint32_t kb[NB], const bool act[NB], uint32_t r[NB],
                                           uint32_t* __restrict__ counts) {
    static_assert(kRankWin % BLOCK == 0, "window entries per thread");
    constexpr int PER = kRankWin / BLOCK;
    __shared__ uint32_t s_cnt[kRankWin];
    __shared__ uint32_t s_k0;
    const int tid = threadIdx.x;
    uint32_t kmin = 0xffffffffu;
#pragma unroll
    for (int b = 0; b < NB; ++b)
        if (act[b]) kmin = min(kmin, kb[b]);
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, o, 64));
    if (tid == 0) s_k0 = 0xffffffffu;
#pragma unroll
    for (int i = 0; i < PER; ++i) s_cnt[tid + i * BLOCK] = 0u;
    __syncthreads();
    if ((tid & 63) == 0) atomicMin(&s_k0, kmin);
    __syncthreads();
    const uint32_t k0 = s_k0;
    uint32_t lr[NB];
    bool loc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        loc[b] = act[b] && kb[b] - k0 < (uint32_t)kRankWin;
        lr[b] = loc[b] ? atomicAdd(&s_cnt[kb[b] - k0], 1u) : 0u;
    }
    __syncthreads();
    // each thread owns window entries tid + i BLOCK: read the count, reserve
    // the places, leave the first place in the entry
    uint32_t c[PER], base[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) c[i] = s_cnt[tid + i * BLOCK];
#pragma unroll
    for (int i = 0; i < PER; ++i) base[i] = c[i] ? atomicAdd(&counts[k0 + (uint32_t)(tid + i * BLOCK)], c[i]) : 0u;
#pragma unroll
    for (int i = 0; i < PER; ++i)
        if (c[i]) s_cnt[tid + i * BLOCK] = base[i];
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b)
        r[b] = loc[b] ? s_cnt[kb[b] - k0] + lr[b] : (act[b] ? atomicAdd(&counts[kb[b]], 1u) : 0u);
}

// Beads in sorted order, NB per thread (MODE 1: one): F = sum of the P plane
// partials of each component (non-bonded, ik route) + the stored bond force.
// MODE 0: Euler-Maruyama step.  The centre-of-mass correction subtracts the
//         mean displacement; the forces sum to zero exactly (pairwise bonds;
//         the ik route with the Nyquist derivative zeroed conserves momentum),
//         so that mean is sqrt(2 kT dt/gamma) times the mean noise, from which
//         the k-space pass has already formed the new integer shift (qs_new;
//         on the exact-gradient route k_form_shift, from the noise and force
//         sums).  Each moved bead goes to pout[j] with its exact new bin key
//         and its rank in that bin.
// MODE 2: GJF step, D_{n+1} = a D_n + mob_dt F + noise_amp (xi_n + xi_{n+1})
//         with D_n = gjf_vs u from the half-step velocity u (vin, sorted
//         order); the same shift, key and rank as MODE 0, and the realised
//         displacement (new minus old position, net of the shift) written
//         back as the new half-step velocity to vout[j].
// MODE 1: forces only, times out_sign, written to out[abi id] ([n][3], float
//         or double).
// BATCH (MODE 0): one launch for all members of a batch, 256-bead blocks
// named by the unit map.  NB (MODE 0 and 2): beads per thread, the block
// covering NB * 256 consecutive beads.
template <typename T, int P, int MODE, bool BATCH = false, int NB = 1>
__global__ void __launch_bounds__(256)
    k_update(const uint4* __restrict__ pin, uint4* __restrict__ pout, const T* __restrict__ fbond,
             const T* __restrict__ fpart, const uint32_t* __restrict__ qs_new,
             long long n, Dims d, Phys ph, uint64_t step, void* out, int out_dtype, unsigned parts, double out_sign,
             uint2* __restrict__ kr,
             uint32_t* __restrict__ counts, uint32_t* __restrict__ flag, const uint32_t* __restrict__ qs_old,
             const T* __restrict__ vin, T* __restrict__ vout, const RepDesc* __restrict__ reps,
             const uint32_t* __restrict__ umap, int parity) {
    const int tid = threadIdx.x;
    const bool need_field = MODE != 1 || (parts & 1u);
    const bool need_bond = MODE != 1 || (parts & 2u);
    long long blk = blockIdx.x;
    if constexpr (BATCH) {
        static_assert(MODE == 0 && NB == 1, "batched steps use Euler-Maruyama, one bead per thread");
        const uint32_t e = umap[blockIdx.x];
        const RepDesc& R = reps[e >> 16];
        pin = R.S.pos;
        pout = R.S.pos_tmp;
        fbond = (const T*)R.S.fbond;
        fpart = (const T*)R.S.fpart;
        qs_new = parity ? R.S.qshift : R.S.qshift_next;
        qs_old = parity ? R.S.qshift_next : R.S.qshift;
        n = R.S.n;
        d = R.d;
        ph = R.ph;
        step += R.step0;
        kr = R.S.kr;
        counts = R.S.counts;
        flag = R.S.flag;
        blk = (long long)(e & 0xffffu);
    }
    if constexpr (MODE != 1) {
        // NB beads per thread, 256 apart (each 256-bead chunk is a contiguous
        // run of the sorted order); every load of the thread's beads is issued
        // before any of them is advanced (a lane past the end reads the last
        // bead and discards it)
        if (n <= 0) return;
        uint4 q[NB];
        T f[NB][3], u[NB][3], fp[NB][3][P], xi[NB][3];
        bool act[NB];
        long long jb[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            jb[b] = (blk * NB + b) * 256LL + tid;
            act[b] = jb[b] < n;
            const long long j = act[b] ? jb[b] : n - 1;
            q[b] = pin[j];
            f[b][0] = fbond[4 * j + 0];
            f[b][1] = fbond[4 * j + 1];
            f[b][2] = fbond[4 * j + 2];
            if constexpr (MODE == 2) {
                u[b][0] = vin[4 * j + 0];
                u[b][1] = vin[4 * j + 1];
                u[b][2] = vin[4 * j + 2];
            }
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int c = 0; c < P; ++c) fp[b][a][c] = fpart[((long long)a * P + c) * n + j];
        }
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                T sa = 0;
#pragma unroll
                for (int c = 0; c < P; ++c) sa += fp[b][a][c];
                f[b][a] += sa;
            }
        const uint32_t nsh[3] = {qs_new[0], qs_new[1], qs_new[2]};  // formed before this kernel
        uint32_t kb[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            kb[b] = 0xffffffffu;
            if (!act[b]) continue;
            const long long j = jb[b];
            const double inv_l[3] = {ph.qx, ph.qy, ph.qz};
            const T mob = (T)ph.mob_dt, amp = (T)ph.noise_amp;
            Noise<T>::draw(q[b].w >> 1, step, ph.seed, xi[b]);
            if constexpr (MODE == 2) {
                T xi1[3];
                Noise<T>::draw(q[b].w >> 1, step + 1, ph.seed, xi1);
                xi[b][0] += xi1[0];
                xi[b][1] += xi1[1];
                xi[b][2] += xi1[2];
            }
            long long dq[3] = {0, 0, 0};
            bool bad = false;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                // explicit fused steps: every instantiation rounds alike
                T disp = fma_t(mob, f[b][a], amp * xi[b][a]);
                if constexpr (MODE == 2) disp = fma_t((T)ph.gjf_a, (T)ph.gjf_vs * u[b][a], disp);
                const double sd = (double)disp * inv_l[a];
                if (!(fabs(sd) < 4.0e18)) bad = true;  // also true for NaN
                else dq[a] = llrint(sd);
            }
            if (bad) {
                atomicOr(flag, 1u);
                dq[0] = dq[1] = dq[2] = 0;
            }
            const uint4 qn =
                uint4{q[b].x + (uint32_t)dq[0], q[b].y + (uint32_t)dq[1], q[b].z + (uint32_t)dq[2], q[b].w};
            pout[j] = qn;
            if constexpr (MODE == 2) {
                // realised displacement: dq minus the step's shift (a small integer)
                const double L[3] = {ph.lx, ph.ly, ph.lz};
                const double inv_vs = 1.0 / ph.gjf_vs;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const long long sh = (long long)(int32_t)(nsh[a] - qs_old[a]);
                    vout[4 * j + a] = (T)((double)(dq[a] - sh) * (L[a] * kInvTwo32) * inv_vs);
                }
                vout[4 * j + 3] = (T)0;
            }
            kb[b] = bin_key(qn.y - nsh[1], qn.z - nsh[2], qn.w & 1u, d, P);
        }
        // ranks: Euler-Maruyama moves about a third of the beads to another bin
        // each step, which breaks the wavefront runs of equal keys, so the
        // workgroup aggregates per key; GJF displacements are small (the
        // velocity carries over), the runs stay long and one atomic per run is
        // cheaper
        uint32_t r[NB];
        if constexpr (MODE == 0) {
            block_rank<NB, 256>(kb, act, r, counts);
        } else {
#pragma unroll
            for (int b = 0; b < NB; ++b) r[b] = bin_rank(kb[b], act[b], counts);  // whole wavefronts take part
        }
#pragma unroll
        for (int b = 0; b < NB; ++b)
            if (act[b]) kr[jb[b]] = uint2{kb[b], r[b]};
    } else {
        const long long j = blockIdx.x * 256LL + tid;
        if (j < n) {
            const uint4 q = pin[j];
            const uint32_t id = q.w >> 1;
            T f[3] = {0, 0, 0};
            if (need_bond) {
                f[0] = fbond[4 * j + 0];
                f[1] = fbond[4 * j + 1];
                f[2] = fbond[4 * j + 2];
            }
            if (need_field) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    T sa = 0;
#pragma unroll
                    for (int c = 0; c < P; ++c) sa += fpart[((long long)a * P + c) * n + j];
                    f[a] += sa;
                }
            }
            const T sg = (T)out_sign;
            if (out_dtype == 0) {
                float* o = reinterpret_cast<float*>(out) + 3 * (long long)id;
                o[0] = (float)(sg * f[0]);
                o[1] = (float)(sg * f[1]);
                o[2] = (float)(sg * f[2]);
            } else {
                double* o = reinterpret_cast<double*>(out) + 3 * (long long)id;
                o[0] = (double)(sg * f[0]);
                o[1] = (double)(sg * f[1]);
                o[2] = (double)(sg * f[2]);
            }
        }
    }
}

// ------------------------------------------------------------ counting sort

// bin_start = exclusive prefix sum of counts over tiles of kScanBins bins (one
// per thread group of 4 in a 256-thread workgroup)
// (bin_start[nbins] = total); counts are cleared for the next use.  Tiles are
// claimed in launch order from a 64-bit ticket and combined by a decoupled
// look-back: each tile publishes its aggregate, then its inclusive prefix, in
// one status word {epoch:30, flag:2, value:32} (flag 1 aggregate, 2
// inclusive), so a tile never waits on a later one.  The ticket also yields
// the launch's epoch (ticket / ntiles), which tells this launch's statuses
// from the previous one's without any clearing.  A wait that outlasts
// kScanSpin polls sets flag bit 4 and gives up.
constexpr int kScanSpin = 1 << 22;

__device__ __forceinline__ unsigned long long scan_status(uint32_t epoch, uint32_t flag, uint32_t value) {
    return ((unsigned long long)((epoch << 2) | flag) << 32) | value;
}

//
// BATCH: one launch for all members of a batch; the ticket orders the tiles
// of all members (each member's tiles consecutively in the unit map), so a
// tile still only waits on tiles claimed before it, of its own member.
template <bool BATCH = false>
__global__ void __launch_bounds__(256)
    k_bin_scan(uint32_t* __restrict__ counts, uint32_t* __restrict__ bin_start, int nbins,
               unsigned long long* __restrict__ status, unsigned long long* __restrict__ ticket,
               uint32_t* __restrict__ flag, const RepDesc* __restrict__ reps, const uint32_t* __restrict__ umap) {
    __shared__ uint32_t s_tile, s_excl, s_rep;
    __shared__ uint32_t wsum[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    unsigned ntiles = gridDim.x;
    if (tid == 0) {
        const unsigned long long t = atomicAdd(ticket, 1ull);
        const uint32_t g = (uint32_t)(t % gridDim.x);
        s_excl = (uint32_t)((t / gridDim.x) & 0x3fffffffull);  // epoch, until the prefix is known
        if constexpr (BATCH) {
            const uint32_t e = umap[g];
            s_rep = e >> 16;
            s_tile = e & 0xffffu;
        } else {
            s_tile = g;
        }
    }
    __syncthreads();
    const uint32_t tile = s_tile, epoch = s_excl;
    if constexpr (BATCH) {
        const RepDesc& R = reps[s_rep];
        counts = R.S.counts;
        bin_start = R.S.bin_start;
        nbins = R.S.nbins;
        status = R.S.scan_status;
        flag = R.S.flag;
        ntiles = (unsigned)R.ntiles;
    }
    const int lo = (int)tile * kScanBins + 4 * tid;
    uint4 v = uint4{0u, 0u, 0u, 0u};
    if (lo < nbins) v = *reinterpret_cast<const uint4*>(counts + lo);
    const uint32_t sum = v.x + v.y + v.z + v.w;
    uint32_t inc = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o, 64);
        if (lane >= o) inc += t;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    const uint32_t agg = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    if (wave == 0) {
        uint32_t excl = 0;
        if (tile == 0) {
            if (lane == 0) __hip_atomic_store(&status[0], scan_status(epoch, 2u, agg), __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (lane == 0) __hip_atomic_store(&status[tile], scan_status(epoch, 1u, agg), __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
            int hi = (int)tile - 1;  // nearest predecessor not yet added
            int spins = 0;
            while (true) {
                const int idx = hi - lane;
                uint32_t f = 2u, val = 0u;
                if (idx >= 0) {
                    const unsigned long long st =
                        __hip_atomic_load(&status[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint32_t w = (uint32_t)(st >> 32);
                    f = (w >> 2) == epoch ? (w & 3u) : 0u;
                    val = (uint32_t)st;
                }
                const unsigned long long incl_mask = __ballot(f == 2u);
                const int first = incl_mask ? __ffsll((long long)incl_mask) - 1 : 64;
                const unsigned long long need = first >= 63 ? ~0ull : ((2ull << first) - 1ull);
                if (__ballot(f == 0u) & need) {
                    if (++spins > kScanSpin) {
                        if (lane == 0) atomicOr(flag, 16u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += wave_sum(lane <= first ? val : 0u);
                if (first < 64) break;
                hi -= 64;
            }
            if (lane == 0) __hip_atomic_store(&status[tile], scan_status(epoch, 2u, excl + agg), __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) s_excl = excl;
    }
    __syncthreads();
    uint32_t run = s_excl + inc - sum;
    for (int w = 0; w < wave; ++w) run += wsum[w];
    if (lo < nbins) {
        uint4 o;
        o.x = run;
        o.y = run + v.x;
        o.z = o.y + v.y;
        o.w = o.z + v.z;
        *reinterpret_cast<uint4*>(bin_start + lo) = o;
        *reinterpret_cast<uint4*>(counts + lo) = uint4{0u, 0u, 0u, 0u};
    }
    if (tile == ntiles - 1 && tid == 0) bin_start[nbins] = s_excl + agg;
}

// The Gaussian increments of step `step` (GJF: steps step and step + 1; the
// draws the update takes) of the beads with ABI ids id[c] (valid[c]) of NB
// 256-bead chunks, summed per chunk in 32.32 fixed point (exact for float
// increments, so the total over chunks does not depend on the bead order) into
// out[3 c .. 3 c + 2] for the first nout chunks (the others lie past the last
// bead).  Called by all 256 threads of the block, lane t holding bead t of
// every chunk.
template <typename T, int NB>
__device__ __forceinline__ void noise_sum_chunks(const uint32_t id[NB], const bool valid[NB], const Phys& ph,
                                                 uint64_t step, long long* __restrict__ out, long long nout) {
    __shared__ long long nred[3 * NB * 4];
    long long ns[3 * NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
        ns[3 * c] = ns[3 * c + 1] = ns[3 * c + 2] = 0;
        if (valid[c]) {
            T xi[3];
            Noise<T>::draw(id[c], step, ph.seed, xi);
            if (ph.gjf) {
                T x1[3];
                Noise<T>::draw(id[c], step + 1, ph.seed, x1);
#pragma unroll
                for (int a = 0; a < 3; ++a) xi[a] += x1[a];
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) ns[3 * c + a] = llrint((double)xi[a] * kTwo32);
        }
    }
    block_sum<long long, 3 * NB>(ns, nred, threadIdx.x, 256);
    if (threadIdx.x == 0)
        for (int q = 0; q < 3 * NB; ++q)
            if (q < 3 * nout) out[q] = ns[q];
}

// Noise sums of step `step` per 256-bead block of pos (any order), as the
// scatter of the previous step leaves them; for the first step of a run.
// BATCH: every member of a batch, bead blocks named by the unit map, at each
// member's own step.
template <typename T, bool BATCH = false>
__global__ void __launch_bounds__(256)
    k_noise_sum(const uint4* __restrict__ pos, long long n, Phys ph, uint64_t step, long long* __restrict__ noise_part,
                const RepDesc* __restrict__ reps, const uint32_t* __restrict__ umap) {
    long long blk = blockIdx.x;
    if constexpr (BATCH) {
        const uint32_t e = umap[blockIdx.x];
        const RepDesc& R = reps[e >> 16];
        pos = R.S.pos;
        n = R.S.n;
        ph = R.ph;
        step = R.step0;
        noise_part = R.S.noise_part;
        blk = (long long)(e & 0xffffu);
    }
    const long long j = blk * 256LL + threadIdx.x;
    const bool valid[1] = {j < n};
    const uint32_t id[1] = {valid[0] ? pos[j].w >> 1 : 0u};
    noise_sum_chunks<T, 1>(id, valid, ph, step, noise_part + 3 * blk, 1);
}

// Move every bead of the previous order to its sorted slot, translate its
// bond partners (slots of the previous order) into sorted slots, and store
// its harmonic bond force F = -2 k_b sum_partners d (d the minimum-image bond
// vector, shift-free in fixed point) as {Fx, Fy, Fz, 0}.  With GJF (vdst not
// null) the half-step velocity moves with the bead.  Single precision: also
// the bead's grid record {x, y, z, id << 1 | species} (grid_record, with the
// current shift qs and order P) to grec[slot].
//
// With noise_part, the block also sums the Gaussian increments of step
// noise_step (GJF: of steps noise_step and noise_step + 1) over each of its
// 256-bead chunks, for the centre-of-mass shift of that step
// (noise_sum_chunks).
//
// NB beads per thread, 256 apart, the block covering NB * 256 consecutive
// beads.  DEG > 0: the partner table (of every member, BATCH) has exactly DEG columns, and the
// partners' slots and positions are held in registers, so the dependent reads
// of all NB beads (key and rank, then bin start) are in flight together;
// DEG == 0: any width, one bead per thread.
template <typename T, bool BATCH = false, int NB = 1, int DEG = 0>
__global__ void __launch_bounds__(256)
    k_scatter(const uint4* __restrict__ pos_tmp, const uint2* __restrict__ kr, const uint32_t* __restrict__ bin_start,
              const int32_t* __restrict__ nbr_src, uint4* __restrict__ pos, int32_t* __restrict__ nbr_dst,
              T* __restrict__ fbond, long long n, int deg, Phys ph, const T* __restrict__ vsrc, T* __restrict__ vdst,
              const RepDesc* __restrict__ reps, const uint32_t* __restrict__ umap, int parity,
              uint4* __restrict__ grec, const uint32_t* __restrict__ qs, Dims d, int P,
              long long* __restrict__ noise_part, uint64_t noise_step) {
    static_assert(DEG > 0 || NB == 1, "a partner table of any width takes one bead per thread");
    // contiguous bead ranges per XCD: bond partners are near in the order
    long long blk = xcd_contiguous(blockIdx.x, gridDim.x);
    if constexpr (BATCH) {
        static_assert(NB == 1, "batched scatter: one bead per thread");
        const uint32_t e = umap[blk];
        const RepDesc& R = reps[e >> 16];
        pos_tmp = R.S.pos_tmp;
        kr = R.S.kr;
        bin_start = R.S.bin_start;
        nbr_src = parity ? R.S.nbr_old : R.S.nbr;
        pos = R.S.pos;
        nbr_dst = parity ? R.S.nbr : R.S.nbr_old;
        fbond = (T*)R.S.fbond;
        n = R.S.n;
        deg = R.S.deg;
        ph = R.ph;
        vsrc = nullptr;
        vdst = nullptr;
        grec = R.S.grec;
        qs = parity ? R.S.qshift : R.S.qshift_next;  // the shift the update of this step formed
        d = R.d;
        noise_part = R.S.noise_part;  // batched steps always sum the next step's noise
        noise_step += R.step0;        // noise_step: the step's index within the batch call, plus one
        blk = (long long)(e & 0xffffu);
    }
    constexpr int DR = DEG > 0 ? DEG : 1;
    long long jb[NB];
    bool act[NB];
    uint2 kj[NB];
    uint4 q[NB];
    int32_t pp[NB][DR];
    // first reads: key and rank, position, partner slots (DEG > 0: a lane past
    // the end reads the last bead and discards it)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        jb[b] = (blk * NB + b) * 256LL + threadIdx.x;
        act[b] = jb[b] < n;
        kj[b] = uint2{0u, 0u};
        q[b] = uint4{0u, 0u, 0u, 0u};
#pragma unroll
        for (int e = 0; e < DR; ++e) pp[b][e] = -1;
        if constexpr (DEG > 0) {
            const long long j = act[b] ? jb[b] : n - 1;
            kj[b] = kr[j];
            q[b] = pos_tmp[j];
#pragma unroll
            for (int e = 0; e < DEG; ++e) pp[b][e] = nbr_src[j * DEG + e];
        } else if (act[b]) {
            kj[b] = kr[jb[b]];
            q[b] = pos_tmp[jb[b]];
        }
    }
    // the block's noise sums, drawn while its reads are in flight
    auto noise_sums = [&]() {
        if (!noise_part) return;
        uint32_t id[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) id[b] = q[b].w >> 1;
        noise_sum_chunks<T, NB>(id, act, ph, noise_step, noise_part + 3 * (blk * NB), (n + 255) / 256 - blk * NB);
    };
    // bond force factors per axis (explicit fused steps below: every
    // instantiation rounds alike)
    const T c = (T)(-2.0 * ph.bond_k);
    const T csx = c * (T)(ph.lx * kInvTwo32), csy = c * (T)(ph.ly * kInvTwo32), csz = c * (T)(ph.lz * kInvTwo32);
    if constexpr (DEG == 0) {
        noise_sums();
        const long long j = jb[0];
        if (!act[0]) return;
        const long long nw = (long long)bin_start[kj[0].x] + kj[0].y;
        const uint4 qj = q[0];
        pos[nw] = qj;
        if constexpr (sizeof(T) == 4)
            grec[nw] = uint4{grid_record(qj.x - qs[0], d.mx, P), grid_record(qj.y - qs[1], d.my, P),
                             grid_record(qj.z - qs[2], d.mz, P), qj.w};
        if (vdst) {
#pragma unroll
            for (int a = 0; a < 4; ++a) vdst[4 * nw + a] = vsrc[4 * j + a];
        }
        T f[3] = {0, 0, 0};
        for (int b = 0; b < deg; ++b) {
            const int p = nbr_src[j * deg + b];
            int32_t np_ = -1;
            if (p >= 0) {
                const uint2 kp = kr[p];
                np_ = (int32_t)(bin_start[kp.x] + kp.y);
                const uint4 qp = pos_tmp[p];
                f[0] = fma_t(csx, (T)fixed_delta(qj.x, qp.x), f[0]);
                f[1] = fma_t(csy, (T)fixed_delta(qj.y, qp.y), f[1]);
                f[2] = fma_t(csz, (T)fixed_delta(qj.z, qp.z), f[2]);
            }
            nbr_dst[nw * deg + b] = np_;
        }
        fbond[4 * nw + 0] = f[0];
        fbond[4 * nw + 1] = f[1];
        fbond[4 * nw + 2] = f[2];
        fbond[4 * nw + 3] = (T)0;
    } else {
        // second reads: own bin start, partners' keys, ranks and positions (a
        // missing partner reads the bead itself)
        uint32_t bs[NB];
        uint2 kp[NB][DEG];
        uint4 qp[NB][DEG];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const long long j = act[b] ? jb[b] : n - 1;
            bs[b] = bin_start[kj[b].x];
#pragma unroll
            for (int e = 0; e < DEG; ++e) {
                const long long p = pp[b][e] >= 0 ? (long long)pp[b][e] : j;
                kp[b][e] = kr[p];
                qp[b][e] = pos_tmp[p];
            }
        }
        noise_sums();
        // third reads: the partners' bin starts
        int32_t np_[NB][DEG];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int e = 0; e < DEG; ++e) {
                const int32_t s0 = (int32_t)(bin_start[kp[b][e].x] + kp[b][e].y);
                np_[b][e] = pp[b][e] >= 0 ? s0 : -1;
            }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (!act[b]) continue;
            const long long j = jb[b], nw = (long long)bs[b] + kj[b].y;
            const uint4 qj = q[b];
            pos[nw] = qj;
            if constexpr (sizeof(T) == 4)
                grec[nw] = uint4{grid_record(qj.x - qs[0], d.mx, P), grid_record(qj.y - qs[1], d.my, P),
                                 grid_record(qj.z - qs[2], d.mz, P), qj.w};
            if (vdst) {
#pragma unroll
                for (int a = 0; a < 4; ++a) vdst[4 * nw + a] = vsrc[4 * j + a];
            }
            T f[3] = {0, 0, 0};
#pragma unroll
            for (int e = 0; e < DEG; ++e) {
                if (pp[b][e] >= 0) {
                    f[0] = fma_t(csx, (T)fixed_delta(qj.x, qp[b][e].x), f[0]);
                    f[1] = fma_t(csy, (T)fixed_delta(qj.y, qp[b][e].y), f[1]);
                    f[2] = fma_t(csz, (T)fixed_delta(qj.z, qp[b][e].z), f[2]);
                }
                nbr_dst[nw * DEG + e] = np_[b][e];
            }
            fbond[4 * nw + 0] = f[0];
            fbond[4 * nw + 1] = f[1];
            fbond[4 * nw + 2] = f[2];
            fbond[4 * nw + 3] = (T)0;
        }
    }
}

// ------------------------------------------------------------ positions I/O

// ABI-order coordinates -> fixed point in pos_tmp with keys and ranks; the
// global shift restarts at zero.
template <typename TI>
__global__ void __launch_bounds__(256)
    k_place(const TI* __restrict__ xyz, const uint32_t* __restrict__ types, uint4* __restrict__ pos_tmp,
            uint2* __restrict__ kr, uint32_t* __restrict__ counts,
            uint32_t* __restrict__ qs, long long n, Dims d, int P, uint32_t* __restrict__ flag) {
    const long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i == 0) qs[0] = qs[1] = qs[2] = qs[3] = 0u;
    if (i >= n) return;
    const double L[3] = {d.lx, d.ly, d.lz};
    uint32_t q[3];
    for (int a = 0; a < 3; ++a) {
        const double x = (double)xyz[3 * i + a];
        if (!isfinite(x)) {
            atomicOr(flag, 1u);
            q[a] = 0u;
            continue;
        }
        double f = x / L[a];
        f -= floor(f);
        q[a] = (uint32_t)(unsigned long long)llrint(f * kTwo32);  // 2^32 wraps to 0
    }
    const uint32_t K = types[i];
    pos_tmp[i] = uint4{q[0], q[1], q[2], ((uint32_t)i << 1) | K};
    const uint32_t kb = bin_key(q[1], q[2], K, d, P);
    kr[i] = uint2{kb, atomicAdd(&counts[kb], 1u)};
}

// GJF half-step velocities between ABI order ([n][3], TA) and sorted order
// ([n][4], T): OP 0 sorted <- ABI, OP 1 ABI <- sorted, OP 2 vtmp[4 id] <-
// sorted (the order k_place gives pos_tmp).
template <typename T, typename TA, int OP>
__global__ void __launch_bounds__(256) k_velocities(const uint4* __restrict__ pos, T* __restrict__ vel,
                                                    T* __restrict__ vtmp, TA* __restrict__ abi, long long n) {
    const long long j = blockIdx.x * 256LL + threadIdx.x;
    if (j >= n) return;
    const long long id = (long long)(pos[j].w >> 1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if constexpr (OP == 0) vel[4 * j + a] = (T)abi[3 * id + a];
        else if constexpr (OP == 1) abi[3 * id + a] = (TA)vel[4 * j + a];
        else vtmp[4 * id + a] = vel[4 * j + a];
    }
    if constexpr (OP == 0) vel[4 * j + 3] = (T)0;
    if constexpr (OP == 2) vtmp[4 * id + 3] = (T)0;
}

template <typename TO>
__global__ void __launch_bounds__(256) k_get_positions(const uint4* __restrict__ pos, const uint32_t* __restrict__ qs,
                                                       long long n, double lx, double ly, double lz,
                                                       TO* __restrict__ xyz) {
    const long long j = blockIdx.x * 256LL + threadIdx.x;
    if (j >= n) return;
    const uint4 q = pos[j];
    const long long id = q.w >> 1;
    xyz[3 * id + 0] = (TO)((double)(q.x - qs[0]) * (lx * kInvTwo32));
    xyz[3 * id + 1] = (TO)((double)(q.y - qs[1]) * (ly * kInvTwo32));
    xyz[3 * id + 2] = (TO)((double)(q.z - qs[2]) * (lz * kInvTwo32));
}


// ============================================================ launchers

// H v accumulation in sorted order: acc = (first ? bond term : acc) + sign * sum of
// the P plane partials per axis; the bond term of U = k_b sum |d|^2 is
// bond_sign 2 k_b sum_partners (v_j - v_p).
template <typename T, int P>
__global__ void __launch_bounds__(256) k_hvp_accum(const T* __restrict__ fpart, long long n,
                                                   const T* __restrict__ vdir, const int32_t* __restrict__ nbr,
                                                   int deg, double bond_k, T* __restrict__ acc, int first, T sign,
                                                   T bond_sign) {
    const long long j = blockIdx.x * 256LL + threadIdx.x;
    if (j >= n) return;
    T r[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T sa = 0;
#pragma unroll
        for (int c = 0; c < P; ++c) sa += fpart[((long long)a * P + c) * n + j];
        r[a] = (first ? (T)0 : acc[4 * j + a]) + sign * sa;
    }
    if (first) {
        const T kb2 = bond_sign * (T)(2.0 * bond_k);
        for (int b = 0; b < deg; ++b) {
            const int p = nbr[j * deg + b];
            if (p < 0) continue;
#pragma unroll
            for (int a = 0; a < 3; ++a) r[a] += kb2 * (vdir[4 * j + a] - vdir[4 * (long long)p + a]);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[4 * j + a] = r[a];
    acc[4 * j + 3] = (T)0;
}

static inline unsigned blocks_for(long long n, int per) { return (unsigned)((n + per - 1) / per); }

// Calls f(std::integral_constant<int, P>{}) for the stencil order P = order.
template <typename F> inline void with_order(int order, F&& f) {
    switch (order) {
        case 1: f(std::integral_constant<int, 1>{}); break;
        case 2: f(std::integral_constant<int, 2>{}); break;
        case 3: f(std::integral_constant<int, 3>{}); break;
        case 4: f(std::integral_constant<int, 4>{}); break;
        case 5: f(std::integral_constant<int, 5>{}); break;
        case 6: f(std::integral_constant<int, 6>{}); break;
        default: f(std::integral_constant<int, 7>{}); break;
    }
}

}  // namespace tild

// HIP kernels of the TILD particle-mesh step for gfx950.
//
// Per step (paper, Sec. "Long-range interactions", Eq. PMM and Fig. pmm):
//   fill_mean   counts grids start at -N_K/M (the mean is carried analytically)
//   spread      c_K(g) += W_i(g) for every bead (order-P B-spline weights)
//   xy_r2c      per z-plane: real-to-complex FFT along x, complex FFT along y
//   z_kmul      per column block: FFT along z, multiply by the smeared
//               chi/kappa kernel, inverse FFT along z of Phi_K and ik_z Phi_K
//   xy_c2r      per z-plane: ik_x, ik_y applied, inverse FFT along y and
//               complex-to-real along x -> the three gradient fields of phi_K
//   gather      F_i = -sum_g W_i(g) grad phi_{s_i}(g), harmonic bonds, Philox
//               noise and the Euler-Maruyama update
#include "tild_kernels.h"

namespace tild {

constexpr int kPairItems = 20;  // row-pair (un)packing items per thread
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
__device__ void block_sum(V* vals, V* scratch /* [NV][nwaves] */, int tid, int nthr) {
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

// ------------------------------------------------------------ fill / spread

template <typename T>
__global__ void __launch_bounds__(256) k_fill_mean(T* __restrict__ dens, long long m, T va, T vb) {
    const long long stride = (long long)gridDim.x * 256;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < 2 * m; i += stride) dens[i] = i < m ? va : vb;
}

template <typename T, int P>
__global__ void __launch_bounds__(256) k_spread_atomic(const uint4* __restrict__ pos, const uint32_t* __restrict__ qs,
                                                       long long n, Dims d, T* __restrict__ dens) {
    const long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= n) return;
    const uint4 q = pos[i];
    int gx, gy, gz;
    T wx[P], wy[P], wz[P];
    assignment_weights<T, P>(q.x - qs[0], d.mx, gx, wx);
    assignment_weights<T, P>(q.y - qs[1], d.my, gy, wy);
    assignment_weights<T, P>(q.z - qs[2], d.mz, gz, wz);
    T* g = dens + (q.w ? d.m : 0);
#pragma unroll
    for (int c = 0; c < P; ++c) {
        int z = gz + c;
        if (z >= d.mz) z -= d.mz;
#pragma unroll
        for (int b = 0; b < P; ++b) {
            int y = gy + b;
            if (y >= d.my) y -= d.my;
            T* row = g + ((long long)z * d.my + y) * d.mx;
            const T wzy = wz[c] * wy[b];
#pragma unroll
            for (int a = 0; a < P; ++a) {
                int x = gx + a;
                if (x >= d.mx) x -= d.mx;
                unsafeAtomicAdd(row + x, wzy * wx[a]);
            }
        }
    }
}

// ------------------------------------------------------------ xy plane passes

// Forward: real plane c[y][x] -> half spectrum H[ky][kx], kx = 0 .. mx/2.
// Rows 2p and 2p+1 are transformed together as one complex row
// z = c_2p + i c_2p+1, then separated with Z(-k)* symmetry.
template <typename T, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_xy_r2c(const T* __restrict__ dens, cplx<T>* __restrict__ spec, Dims d,
                                                  FftPlan px, FftPlan py, const cplx<T>* __restrict__ tw) {
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    C* S = reinterpret_cast<C*>(smem);
    const int tid = threadIdx.x;
    const int z = blockIdx.x, K = blockIdx.y;
    const int mx = d.mx, my = d.my, hx = d.hx, np = d.npair;
    const T* src = dens + ((long long)K * d.mz + z) * (long long)my * mx;
    for (int i = tid; i < np * mx; i += BLOCK) {
        const int p = i / mx, x = i - p * mx;
        const T re = src[(2 * p) * mx + x];
        const T im = (2 * p + 1 < my) ? src[(2 * p + 1) * mx + x] : (T)0;
        S[i] = C{re, im};
    }
    __syncthreads();
    fft_lines<C, 0>(S, LineMap{np, np, mx, 0, 1}, px, tw, tid, BLOCK);
    C ra[kPairItems], rb[kPairItems];
    const int items = np * hx;
#pragma unroll
    for (int u = 0; u < kPairItems; ++u) {
        const int i = tid + u * BLOCK;
        if (i < items) {
            const int p = i / hx, kx = i - p * hx;
            const C a = S[p * mx + kx];
            const C b = S[p * mx + (kx == 0 ? 0 : mx - kx)];
            ra[u] = C{(T)0.5 * (a.x + b.x), (T)0.5 * (a.y - b.y)};
            rb[u] = C{(T)0.5 * (a.y + b.y), (T)0.5 * (b.x - a.x)};
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPairItems; ++u) {
        const int i = tid + u * BLOCK;
        if (i < items) {
            const int p = i / hx, kx = i - p * hx;
            S[(2 * p) * hx + kx] = ra[u];
            if (2 * p + 1 < my) S[(2 * p + 1) * hx + kx] = rb[u];
        }
    }
    __syncthreads();
    fft_lines<C, 0>(S, LineMap{hx, hx, 1, 0, hx}, py, tw, tid, BLOCK);
    C* dst = spec + ((long long)K * d.mz + z) * d.hplane;
    for (int i = tid; i < my * hx; i += BLOCK) dst[i] = S[i];
}

// Inverse: for a = x, y, z build the half spectrum of d_a phi_K on plane z,
// inverse FFT along y, then complex-to-real along x with rows 2p and 2p+1
// carried as the real and imaginary parts of one complex row.
template <typename T, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_xy_c2r(const cplx<T>* __restrict__ zout, T* __restrict__ grad, Dims d,
                                                  FftPlan px, FftPlan py, const cplx<T>* __restrict__ tw, Phys ph) {
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    C* S = reinterpret_cast<C*>(smem);
    const int tid = threadIdx.x;
    const int z = blockIdx.x, K = blockIdx.y;
    const int mx = d.mx, my = d.my, hx = d.hx, np = d.npair;
    const T kfx = (T)(kTwoPi / ph.lx), kfy = (T)(kTwoPi / ph.ly);
    for (int a = 0; a < 3; ++a) {
        const C* src = zout + ((long long)(a < 2 ? K : 2 + K) * d.mz + z) * d.hplane;
        for (int i = tid; i < my * hx; i += BLOCK) {
            const int ky = i / hx, kx = i - ky * hx;
            C v = src[i];
            if (a == 0) {
                const T k = (2 * kx == mx) ? (T)0 : kfx * (T)kx;
                v = C{-k * v.y, k * v.x};
            } else if (a == 1) {
                const int ny = ky > my / 2 ? ky - my : ky;
                const T k = (2 * ky == my) ? (T)0 : kfy * (T)ny;
                v = C{-k * v.y, k * v.x};
            }
            S[i] = v;
        }
        __syncthreads();
        fft_lines<C, 1>(S, LineMap{hx, hx, 1, 0, hx}, py, tw, tid, BLOCK);
        C rz[kPairItems];
        const int items = np * mx;
#pragma unroll
        for (int u = 0; u < kPairItems; ++u) {
            const int i = tid + u * BLOCK;
            if (i < items) {
                const int p = i / mx, x = i - p * mx;
                C A, B;
                if (x < hx) {
                    A = S[(2 * p) * hx + x];
                    B = (2 * p + 1 < my) ? S[(2 * p + 1) * hx + x] : C{0, 0};
                } else {
                    const int xs = mx - x;
                    const C a0 = S[(2 * p) * hx + xs];
                    const C b0 = (2 * p + 1 < my) ? S[(2 * p + 1) * hx + xs] : C{0, 0};
                    A = C{a0.x, -a0.y};
                    B = C{b0.x, -b0.y};
                }
                rz[u] = C{A.x - B.y, A.y + B.x};
            }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kPairItems; ++u) {
            const int i = tid + u * BLOCK;
            if (i < items) S[i] = rz[u];
        }
        __syncthreads();
        fft_lines<C, 1>(S, LineMap{np, np, mx, 0, 1}, px, tw, tid, BLOCK);
        T* dst = grad + (((long long)K * 3 + a) * d.mz + z) * (long long)my * mx;
        for (int i = tid; i < items; i += BLOCK) {
            const int p = i / mx, x = i - p * mx;
            const C v = S[i];
            dst[(2 * p) * mx + x] = v.x;
            if (2 * p + 1 < my) dst[(2 * p + 1) * mx + x] = v.y;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ z pass + k-space multiply

// Column block c0 .. c0+cb-1 of the flattened (ky, kx) half-spectrum plane,
// all z.  After the forward z FFT the spectra c^_A, c^_B become
//   Phi^_K = (u^/N) sum_L eps_KL c^_L,  eps_AA = eps_BB = kappa, eps_AB = chi + kappa,
// with u^ = exp(-a^2 k^2) (zero at k = 0: the k = 0 field has no gradient),
// and both Phi^_K and ik_z Phi^_K are transformed back along z.  With
// `want_energy` the block also accumulates, in float64 over the half
// spectrum (weight 2 for kx strictly between 0 and mx/2):
//   sum u^ Re(c^_A* c^_B), sum_{k!=0} u^ |c^_A + c^_B|^2 and, per axis,
//   sum k_a^2 u^ [(chi/N) Re(c^_A* c^_B) + (kappa/2N) |c^_+|^2].
template <typename T, int BLOCK, int ENERGY_ONLY>
__global__ void __launch_bounds__(BLOCK) k_z_kmul(const cplx<T>* __restrict__ spec, cplx<T>* __restrict__ zout, Dims d,
                                                  FftPlan pz, const cplx<T>* __restrict__ tw, Phys ph, int cb,
                                                  double* __restrict__ epart, int want_energy) {
    using C = cplx<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[5 * (BLOCK / 64)];
    C* b0 = reinterpret_cast<C*>(smem);
    const int tid = threadIdx.x;
    const int mz = d.mz, my = d.my, mx = d.mx, hx = d.hx;
    const int cbp = cb + 1;
    C* b1 = b0 + 2 * mz * cbp;
    const long long cn = d.hplane;
    const long long c0 = (long long)blockIdx.x * cb;
    for (int i = tid; i < 2 * mz * cb; i += BLOCK) {
        const int K = i / (mz * cb);
        const int r = i - K * mz * cb;
        const int z = r / cb, j = r - z * cb;
        const long long c = c0 + j;
        b0[(K * mz + z) * cbp + j] = c < cn ? spec[((long long)K * mz + z) * cn + c] : C{0, 0};
    }
    __syncthreads();
    fft_lines<C, 0>(b0, LineMap{2 * cb, cb, 1, mz * cbp, cbp}, pz, tw, tid, BLOCK);

    double acc[5] = {0, 0, 0, 0, 0};
    const double kfx = kTwoPi / ph.lx, kfy = kTwoPi / ph.ly, kfz = kTwoPi / ph.lz;
    const T a2 = (T)ph.a2, inv_n = (T)ph.inv_n, kap = (T)ph.kappa, cpk = (T)(ph.chi + ph.kappa);
    for (int i = tid; i < mz * cb; i += BLOCK) {
        const int z = i / cb, j = i - z * cb;
        const long long c = c0 + j;
        const C A = b0[z * cbp + j], B = b0[(mz + z) * cbp + j];
        C PA{0, 0}, PB{0, 0}, QA{0, 0}, QB{0, 0};
        if (c < cn) {
            const int ky = (int)(c / hx), kx = (int)(c - (long long)ky * hx);
            const int ny = ky > my / 2 ? ky - my : ky;
            const int nz = z > mz / 2 ? z - mz : z;
            if (kx != 0 || ny != 0 || nz != 0) {
                const T kxv = (T)(kfx * kx), kyv = (T)(kfy * ny), kzv = (T)(kfz * nz);
                const T k2 = kxv * kxv + kyv * kyv + kzv * kzv;
                const T f = exp(-a2 * k2) * inv_n;
                PA = C{f * (kap * A.x + cpk * B.x), f * (kap * A.y + cpk * B.y)};
                PB = C{f * (cpk * A.x + kap * B.x), f * (cpk * A.y + kap * B.y)};
                const T kzd = (2 * z == mz) ? (T)0 : kzv;
                QA = C{-kzd * PA.y, kzd * PA.x};
                QB = C{-kzd * PB.y, kzd * PB.x};
                if (want_energy) {
                    const double w = (kx == 0 || 2 * kx == mx) ? 1.0 : 2.0;
                    const double dkx = kfx * kx, dky = kfy * ny, dkz = kfz * nz;
                    const double uh = w * ::exp(-ph.a2 * (dkx * dkx + dky * dky + dkz * dkz));
                    const double cross = (double)A.x * B.x + (double)A.y * B.y;
                    const double sx = (double)A.x + B.x, sy = (double)A.y + B.y;
                    const double plus = sx * sx + sy * sy;
                    const double core = uh * (ph.chi * ph.inv_n * cross + 0.5 * ph.kappa * ph.inv_n * plus);
                    acc[0] += uh * cross;
                    acc[1] += uh * plus;
                    acc[2] += dkx * dkx * core;
                    acc[3] += dky * dky * core;
                    acc[4] += dkz * dkz * core;
                }
            } else if (want_energy) {
                // k = 0 of the mean-subtracted counts is zero; the constant
                // chi N_A N_B / N is added when the partials are reduced.
            }
        }
        if (!ENERGY_ONLY) {
            b0[z * cbp + j] = PA;
            b0[(mz + z) * cbp + j] = PB;
            b1[z * cbp + j] = QA;
            b1[(mz + z) * cbp + j] = QB;
        }
    }
    if (want_energy) {
        block_sum<double, 5>(acc, red, tid, BLOCK);
        if (tid == 0)
            for (int q = 0; q < 5; ++q) epart[blockIdx.x * 5 + q] = acc[q];
    }
    if (ENERGY_ONLY) return;
    __syncthreads();
    fft_lines<C, 1>(b0, LineMap{4 * cb, cb, 1, mz * cbp, cbp}, pz, tw, tid, BLOCK);
    for (int i = tid; i < 4 * mz * cb; i += BLOCK) {
        const int q = i / (mz * cb);
        const int r = i - q * mz * cb;
        const int z = r / cb, j = r - z * cb;
        const long long c = c0 + j;
        if (c < cn) zout[((long long)q * mz + z) * cn + c] = b0[(q * mz + z) * cbp + j];
    }
}

// ------------------------------------------------------------ gather + bonds + update

// MODE 0: one Euler-Maruyama step, positions pin -> pout, global shift
//         qs_in -> qs_out (centre-of-mass correction by the last block).
// MODE 1: forces only, written to `out` ([n][3], float or double).
template <typename T, int P, int MODE>
__global__ void __launch_bounds__(256)
    k_gather(const uint4* __restrict__ pin, uint4* __restrict__ pout, const uint32_t* __restrict__ qs_in,
             uint32_t* __restrict__ qs_out, long long n, Dims d, const T* __restrict__ grad,
             const int32_t* __restrict__ boff, const int32_t* __restrict__ bnbr, Phys ph, uint64_t step, void* out,
             int out_dtype, unsigned parts, unsigned long long* __restrict__ com_acc, uint32_t* __restrict__ flag) {
    __shared__ long long red[3 * 4];
    const int tid = threadIdx.x;
    const long long i = blockIdx.x * 256LL + tid;
    long long dq[3] = {0, 0, 0};
    const uint32_t s0 = qs_in[0], s1 = qs_in[1], s2 = qs_in[2];
    if (i < n) {
        const uint4 q = pin[i];
        T fn[3] = {0, 0, 0}, fb[3] = {0, 0, 0};
        if (MODE == 0 || (parts & 1u)) {
            int gx, gy, gz;
            T wx[P], wy[P], wz[P];
            assignment_weights<T, P>(q.x - s0, d.mx, gx, wx);
            assignment_weights<T, P>(q.y - s1, d.my, gy, wy);
            assignment_weights<T, P>(q.z - s2, d.mz, gz, wz);
            const T* gf = grad + (long long)q.w * 3 * d.m;
#pragma unroll
            for (int c = 0; c < P; ++c) {
                int z = gz + c;
                if (z >= d.mz) z -= d.mz;
#pragma unroll
                for (int b = 0; b < P; ++b) {
                    int y = gy + b;
                    if (y >= d.my) y -= d.my;
                    const long long row = ((long long)z * d.my + y) * d.mx;
                    const T wzy = wz[c] * wy[b];
#pragma unroll
                    for (int a = 0; a < P; ++a) {
                        int x = gx + a;
                        if (x >= d.mx) x -= d.mx;
                        const T w = wzy * wx[a];
                        const long long g = row + x;
                        fn[0] -= w * gf[g];
                        fn[1] -= w * gf[d.m + g];
                        fn[2] -= w * gf[2 * d.m + g];
                    }
                }
            }
        }
        if (MODE == 0 || (parts & 2u)) {
            const T sx = (T)(ph.lx * kInvTwo32), sy = (T)(ph.ly * kInvTwo32), sz = (T)(ph.lz * kInvTwo32);
            const T k2 = (T)(2.0 * ph.bond_k);
            const int jb = boff[i], je = boff[i + 1];
            for (int j = jb; j < je; ++j) {
                const uint4 p = pin[bnbr[j]];
                fb[0] -= k2 * sx * (T)fixed_delta(q.x, p.x);
                fb[1] -= k2 * sy * (T)fixed_delta(q.y, p.y);
                fb[2] -= k2 * sz * (T)fixed_delta(q.z, p.z);
            }
        }
        if (MODE == 1) {
            T f[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) f[a] = ((parts & 1u) ? fn[a] : (T)0) + ((parts & 2u) ? fb[a] : (T)0);
            if (out_dtype == 0) {
                float* o = reinterpret_cast<float*>(out) + 3 * i;
                o[0] = (float)f[0];
                o[1] = (float)f[1];
                o[2] = (float)f[2];
            } else {
                double* o = reinterpret_cast<double*>(out) + 3 * i;
                o[0] = (double)f[0];
                o[1] = (double)f[1];
                o[2] = (double)f[2];
            }
        } else {
            T xi[3];
            Noise<T>::draw((uint32_t)i, step, ph.seed, xi);
            const double inv_l[3] = {kTwo32 / ph.lx, kTwo32 / ph.ly, kTwo32 / ph.lz};
            const T mob = (T)ph.mob_dt, amp = (T)ph.noise_amp;
            bool bad = false;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const T disp = mob * (fn[a] + fb[a]) + amp * xi[a];
                const double s = (double)disp * inv_l[a];
                if (!(fabs(s) < 4.0e18)) {  // also false for NaN
                    bad = true;
                } else {
                    dq[a] = llrint(s);
                }
            }
            if (bad) {
                atomicOr(flag, 1u);
                dq[0] = dq[1] = dq[2] = 0;
            }
            pout[i] = uint4{q.x + (uint32_t)dq[0], q.y + (uint32_t)dq[1], q.z + (uint32_t)dq[2], q.w};
        }
    }
    if (MODE == 0) {
        // Exact integer sum of the applied displacements; the last block to
        // finish turns it into the new global shift.
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            long long v = wave_sum(dq[a]);
            if ((tid & 63) == 0) red[a * 4 + (tid >> 6)] = v;
        }
        __syncthreads();
        if (tid == 0) {
            for (int a = 0; a < 3; ++a) {
                const long long s = red[a * 4] + red[a * 4 + 1] + red[a * 4 + 2] + red[a * 4 + 3];
                atomicAdd(&com_acc[a], (unsigned long long)s);
            }
            __threadfence();
            const unsigned long long ticket = atomicAdd(&com_acc[3], 1ull);
            if (ticket == (unsigned long long)gridDim.x - 1) {
                __threadfence();
                const uint32_t sh[3] = {s0, s1, s2};
                for (int a = 0; a < 3; ++a) {
                    const long long tot = (long long)atomicAdd(&com_acc[a], 0ull);
                    long long shift = 0;
                    if (ph.com_correct) shift = llround((double)tot / (double)n);
                    qs_out[a] = sh[a] + (uint32_t)shift;
                    com_acc[a] = 0ull;
                }
                qs_out[3] = 0u;
                com_acc[3] = 0ull;
            }
        }
    }
}

// Bond energy and virial: E = k_b sum |d|^2, W_aa = -2 k_b sum d_a^2 (each
// bond is visited from both ends, hence the factor 1/2).
__global__ void __launch_bounds__(256) k_bond_energy(const uint4* __restrict__ pin, long long n,
                                                     const int32_t* __restrict__ boff,
                                                     const int32_t* __restrict__ bnbr, Phys ph,
                                                     double* __restrict__ bpart) {
    __shared__ double red[4 * 4];
    const int tid = threadIdx.x;
    const long long i = blockIdx.x * 256LL + tid;
    double acc[4] = {0, 0, 0, 0};
    if (i < n) {
        const uint4 q = pin[i];
        const double sx = ph.lx * kInvTwo32, sy = ph.ly * kInvTwo32, sz = ph.lz * kInvTwo32;
        for (int j = boff[i]; j < boff[i + 1]; ++j) {
            const uint4 p = pin[bnbr[j]];
            const double dx = sx * fixed_delta(q.x, p.x), dy = sy * fixed_delta(q.y, p.y),
                         dz = sz * fixed_delta(q.z, p.z);
            acc[0] += 0.5 * ph.bond_k * (dx * dx + dy * dy + dz * dz);
            acc[1] -= ph.bond_k * dx * dx;
            acc[2] -= ph.bond_k * dy * dy;
            acc[3] -= ph.bond_k * dz * dz;
        }
    }
    block_sum<double, 4>(acc, red, tid, 256);
    if (tid == 0)
        for (int q = 0; q < 4; ++q) bpart[blockIdx.x * 4 + q] = acc[q];
}

// Deterministic final sum (fixed order) of the energy partials.
__global__ void __launch_bounds__(256) k_reduce_energy(const double* __restrict__ epart, int nz,
                                                       const double* __restrict__ bpart, int nb, Phys ph,
                                                       double n_a, double n_b, double* __restrict__ eout) {
    __shared__ double red[9 * 4];
    const int tid = threadIdx.x;
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = tid; i < nz; i += 256)
        for (int q = 0; q < 5; ++q) acc[q] += epart[i * 5 + q];
    for (int i = tid; i < nb; i += 256)
        for (int q = 0; q < 4; ++q) acc[5 + q] += bpart[i * 4 + q];
    block_sum<double, 9>(acc, red, tid, 256);
    if (tid == 0) {
        const double e_chi = ph.chi * ph.inv_n * acc[0] + ph.chi * n_a * n_b * ph.inv_n;
        const double e_kap = 0.5 * ph.kappa * ph.inv_n * acc[1];
        const double e_b = acc[5];
        eout[0] = e_b;
        eout[1] = e_chi;
        eout[2] = e_kap;
        eout[3] = e_b + e_chi + e_kap;
        for (int a = 0; a < 3; ++a) eout[4 + a] = -2.0 * ph.a2 * acc[2 + a] + acc[6 + a];
        eout[7] = 0.0;
    }
}

// ------------------------------------------------------------ positions I/O

template <typename TI>
__global__ void __launch_bounds__(256) k_set_positions(const TI* __restrict__ xyz, uint4* __restrict__ pos,
                                                       uint32_t* __restrict__ qs, long long n, double lx, double ly,
                                                       double lz, uint32_t* __restrict__ flag) {
    const long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i == 0) qs[0] = qs[1] = qs[2] = qs[3] = 0u;
    if (i >= n) return;
    const double L[3] = {lx, ly, lz};
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
    const uint4 old = pos[i];
    pos[i] = uint4{q[0], q[1], q[2], old.w};
}

template <typename TO>
__global__ void __launch_bounds__(256) k_get_positions(const uint4* __restrict__ pos, const uint32_t* __restrict__ qs,
                                                       long long n, double lx, double ly, double lz,
                                                       TO* __restrict__ xyz) {
    const long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= n) return;
    const uint4 q = pos[i];
    xyz[3 * i + 0] = (TO)((double)(q.x - qs[0]) * (lx * kInvTwo32));
    xyz[3 * i + 1] = (TO)((double)(q.y - qs[1]) * (ly * kInvTwo32));
    xyz[3 * i + 2] = (TO)((double)(q.z - qs[2]) * (lz * kInvTwo32));
}

__global__ void __launch_bounds__(256) k_stream_copy(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                     long long n16) {
    const long long stride = (long long)gridDim.x * 256;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

// ============================================================ launchers

static inline unsigned blocks_for(long long n, int per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_fill_mean(const Launch& L, DeviceState& S) {
    const double va = -(double)S.n_a / (double)L.d.m, vb = -(double)S.n_b / (double)L.d.m;
    const unsigned g = (unsigned)std::min<long long>(blocks_for(2 * L.d.m, 256), 4096);
    if (L.precision == 0)
        hipLaunchKernelGGL(k_fill_mean<float>, dim3(g), dim3(256), 0, L.stream, (float*)S.dens, L.d.m, (float)va,
                           (float)vb);
    else
        hipLaunchKernelGGL(k_fill_mean<double>, dim3(g), dim3(256), 0, L.stream, (double*)S.dens, L.d.m, va, vb);
    return hipGetLastError();
}

template <typename T, int P> static void spread_p(const Launch& L, DeviceState& S, const uint32_t* qs) {
    hipLaunchKernelGGL((k_spread_atomic<T, P>), dim3(blocks_for(S.n, 256)), dim3(256), 0, L.stream, S.pos, qs, S.n,
                       L.d, (T*)S.dens);
}

template <typename T> static void spread_t(const Launch& L, DeviceState& S, const uint32_t* qs) {
    switch (L.order) {
        case 1: spread_p<T, 1>(L, S, qs); break;
        case 2: spread_p<T, 2>(L, S, qs); break;
        case 3: spread_p<T, 3>(L, S, qs); break;
        case 4: spread_p<T, 4>(L, S, qs); break;
        case 5: spread_p<T, 5>(L, S, qs); break;
        case 6: spread_p<T, 6>(L, S, qs); break;
        default: spread_p<T, 7>(L, S, qs); break;
    }
}

hipError_t launch_spread(const Launch& L, DeviceState& S) {
    if (S.n == 0) return hipSuccess;
    if (L.precision == 0) spread_t<float>(L, S, S.qshift);
    else spread_t<double>(L, S, S.qshift);
    return hipGetLastError();
}

size_t plane_lds_bytes(const Launch& L) {
    const size_t c = L.precision == 0 ? sizeof(float2) : sizeof(double2);
    const size_t a = (size_t)L.d.npair * L.d.mx, b = (size_t)L.d.my * L.d.hx;
    return c * (a > b ? a : b);
}

size_t z_lds_bytes(const Launch& L) {
    const size_t c = L.precision == 0 ? sizeof(float2) : sizeof(double2);
    return c * 4 * (size_t)L.d.mz * (size_t)(L.z_cols + 1);
}

template <typename T, int B> static void xy_r2c_b(const Launch& L, DeviceState& S) {
    hipLaunchKernelGGL((k_xy_r2c<T, B>), dim3(L.d.mz, 2), dim3(B), plane_lds_bytes(L), L.stream, (const T*)S.dens,
                       (cplx<T>*)S.spec, L.d, L.px, L.py, (const cplx<T>*)S.tw);
}
template <typename T, int B> static void xy_c2r_b(const Launch& L, DeviceState& S) {
    hipLaunchKernelGGL((k_xy_c2r<T, B>), dim3(L.d.mz, 2), dim3(B), plane_lds_bytes(L), L.stream,
                       (const cplx<T>*)S.zout, (T*)S.grad, L.d, L.px, L.py, (const cplx<T>*)S.tw, L.ph);
}

hipError_t launch_xy_r2c(const Launch& L, DeviceState& S) {
    if (L.precision == 0) {
        if (L.plane_block == 256) xy_r2c_b<float, 256>(L, S);
        else if (L.plane_block == 512) xy_r2c_b<float, 512>(L, S);
        else xy_r2c_b<float, 1024>(L, S);
    } else {
        if (L.plane_block == 256) xy_r2c_b<double, 256>(L, S);
        else xy_r2c_b<double, 512>(L, S);
    }
    return hipGetLastError();
}

hipError_t launch_xy_c2r(const Launch& L, DeviceState& S) {
    if (L.precision == 0) {
        if (L.plane_block == 256) xy_c2r_b<float, 256>(L, S);
        else if (L.plane_block == 512) xy_c2r_b<float, 512>(L, S);
        else xy_c2r_b<float, 1024>(L, S);
    } else {
        if (L.plane_block == 256) xy_c2r_b<double, 256>(L, S);
        else xy_c2r_b<double, 512>(L, S);
    }
    return hipGetLastError();
}

template <typename T, int EO> static void z_t(const Launch& L, DeviceState& S, int want_energy) {
    hipLaunchKernelGGL((k_z_kmul<T, 256, EO>), dim3(L.n_zblocks), dim3(256), z_lds_bytes(L), L.stream,
                       (const cplx<T>*)S.spec, (cplx<T>*)S.zout, L.d, L.pz, (const cplx<T>*)S.tw, L.ph, L.z_cols,
                       S.epart, want_energy);
}

hipError_t launch_z_kmul(const Launch& L, DeviceState& S, bool energy_only) {
    if (L.precision == 0) {
        if (energy_only) z_t<float, 1>(L, S, 1);
        else z_t<float, 0>(L, S, 0);
    } else {
        if (energy_only) z_t<double, 1>(L, S, 1);
        else z_t<double, 0>(L, S, 0);
    }
    return hipGetLastError();
}

template <typename T, int P, int MODE>
static void gather_p(const Launch& L, DeviceState& S, uint64_t step, void* out, int out_dtype, unsigned parts) {
    hipLaunchKernelGGL((k_gather<T, P, MODE>), dim3(blocks_for(S.n, 256)), dim3(256), 0, L.stream, S.pos, S.pos_next,
                       S.qshift, S.qshift_next, S.n, L.d, (const T*)S.grad, S.bond_off, S.bond_nbr, L.ph, step, out,
                       out_dtype, parts, S.com_acc, S.flag);
}

template <typename T, int MODE>
static void gather_t(const Launch& L, DeviceState& S, uint64_t step, void* out, int od, unsigned parts) {
    switch (L.order) {
        case 1: gather_p<T, 1, MODE>(L, S, step, out, od, parts); break;
        case 2: gather_p<T, 2, MODE>(L, S, step, out, od, parts); break;
        case 3: gather_p<T, 3, MODE>(L, S, step, out, od, parts); break;
        case 4: gather_p<T, 4, MODE>(L, S, step, out, od, parts); break;
        case 5: gather_p<T, 5, MODE>(L, S, step, out, od, parts); break;
        case 6: gather_p<T, 6, MODE>(L, S, step, out, od, parts); break;
        default: gather_p<T, 7, MODE>(L, S, step, out, od, parts); break;
    }
}

hipError_t launch_gather(const Launch& L, DeviceState& S, int mode, uint64_t step, void* out, int out_dtype,
                         unsigned parts) {
    if (S.n == 0) return hipSuccess;
    if (L.precision == 0) {
        if (mode == 0) gather_t<float, 0>(L, S, step, out, out_dtype, parts);
        else gather_t<float, 1>(L, S, step, out, out_dtype, parts);
    } else {
        if (mode == 0) gather_t<double, 0>(L, S, step, out, out_dtype, parts);
        else gather_t<double, 1>(L, S, step, out, out_dtype, parts);
    }
    return hipGetLastError();
}

hipError_t launch_bond_energy(const Launch& L, DeviceState& S) {
    hipLaunchKernelGGL(k_bond_energy, dim3(L.n_bblocks), dim3(256), 0, L.stream, S.pos, S.n, S.bond_off, S.bond_nbr,
                       L.ph, S.bpart);
    return hipGetLastError();
}

hipError_t launch_reduce_energy(const Launch& L, DeviceState& S) {
    hipLaunchKernelGGL(k_reduce_energy, dim3(1), dim3(256), 0, L.stream, S.epart, L.n_zblocks, S.bpart, L.n_bblocks,
                       L.ph, (double)S.n_a, (double)S.n_b, S.eout);
    return hipGetLastError();
}

hipError_t launch_set_positions(const Launch& L, DeviceState& S, const void* xyz, int dtype) {
    const unsigned g = blocks_for(S.n > 0 ? S.n : 1, 256);
    if (dtype == 0)
        hipLaunchKernelGGL(k_set_positions<float>, dim3(g), dim3(256), 0, L.stream, (const float*)xyz, S.pos,
                           S.qshift, S.n, L.ph.lx, L.ph.ly, L.ph.lz, S.flag);
    else
        hipLaunchKernelGGL(k_set_positions<double>, dim3(g), dim3(256), 0, L.stream, (const double*)xyz, S.pos,
                           S.qshift, S.n, L.ph.lx, L.ph.ly, L.ph.lz, S.flag);
    return hipGetLastError();
}

hipError_t launch_get_positions(const Launch& L, DeviceState& S, void* xyz, int dtype) {
    if (S.n == 0) return hipSuccess;
    const unsigned g = blocks_for(S.n, 256);
    if (dtype == 0)
        hipLaunchKernelGGL(k_get_positions<float>, dim3(g), dim3(256), 0, L.stream, S.pos, S.qshift, S.n, L.ph.lx,
                           L.ph.ly, L.ph.lz, (float*)xyz);
    else
        hipLaunchKernelGGL(k_get_positions<double>, dim3(g), dim3(256), 0, L.stream, S.pos, S.qshift, S.n, L.ph.lx,
                           L.ph.ly, L.ph.lz, (double*)xyz);
    return hipGetLastError();
}

hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t stream) {
    const long long n16 = (long long)(bytes / 16);
    const unsigned g = (unsigned)std::min<long long>(blocks_for(n16 > 0 ? n16 : 1, 256), 16384);
    hipLaunchKernelGGL(k_stream_copy, dim3(g), dim3(256), 0, stream, (uint4*)dst, (const uint4*)src, n16);
    return hipGetLastError();
}

template <typename T, int B> static hipError_t attr_plane(size_t lds) {
    hipError_t e = hipFuncSetAttribute((const void*)k_xy_r2c<T, B>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_xy_c2r<T, B>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t configure_kernel_attributes(const Launch& L) {
    const size_t lp = plane_lds_bytes(L), lz = z_lds_bytes(L);
    hipError_t e = hipSuccess;
    if (L.precision == 0) {
        if (L.plane_block == 256) e = attr_plane<float, 256>(lp);
        else if (L.plane_block == 512) e = attr_plane<float, 512>(lp);
        else e = attr_plane<float, 1024>(lp);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_z_kmul<float, 256, 0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lz);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_z_kmul<float, 256, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lz);
    } else {
        if (L.plane_block == 256) e = attr_plane<double, 256>(lp);
        else e = attr_plane<double, 512>(lp);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_z_kmul<double, 256, 0>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lz);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)k_z_kmul<double, 256, 1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lz);
    }
    return e;
}

}  // namespace tild

// Launchers of the per-step kernels other than the plane passes (k-space pass,
// update, bin scan, scatter, energies, positions, velocities) and the kernel
// attributes; the device code itself is in tild_device.h.
#include "tild_device.h"

namespace tild {

// Exact-gradient route: the non-bonded forces do not sum to zero, so the
// step's centre-of-mass shift comes from the per-block noise sums and the
// per-plane force sums (32.32 fixed point, so the total is order-independent):
// the mean displacement is (sqrt(2 kT dt/gamma) sum xi + (dt/gamma) sum F) / N.
constexpr int kShiftBlock = 1024;  // one workgroup; its threads share the per-block and per-plane partials

__global__ void __launch_bounds__(kShiftBlock) k_form_shift(const long long* __restrict__ noise_part,
                                                            const long long* __restrict__ fsum_part, int nplanes,
                                                            long long n, Phys ph, const uint32_t* __restrict__ qs,
                                                            uint32_t* __restrict__ qs_next) {
    __shared__ long long red[6 * (kShiftBlock / 64)];
    const int tid = threadIdx.x;
    long long v[6] = {0, 0, 0, 0, 0, 0};
    const long long nb = (n + 255) / 256;
    if (nb > 0) noise_total<kShiftBlock>(noise_part, nb, v);
    if (nplanes > 0) noise_total<kShiftBlock>(fsum_part, nplanes, v + 3);
    block_sum<long long, 6>(v, red, tid, kShiftBlock);
    if (tid == 0) {
        const double L[3] = {ph.lx, ph.ly, ph.lz};
        for (int a = 0; a < 3; ++a) {
            long long shift = 0;
            if (ph.com_correct && n > 0) {
                const double mean =
                    (ph.noise_amp * ((double)v[a] * kInvTwo32) + ph.mob_dt * ((double)v[3 + a] * kInvTwo32)) /
                    (double)n;
                shift = llround(mean * (kTwo32 / L[a]));
            }
            qs_next[a] = qs[a] + (uint32_t)shift;
        }
        qs_next[3] = 0u;
    }
}

// Bond energy and virial: E = k_b sum |d|^2, W_aa = -2 k_b sum d_a^2 (each
// bond is visited from both ends, hence the factor 1/2).
__global__ void __launch_bounds__(256) k_bond_energy(const uint4* __restrict__ pin, long long n,
                                                     const int32_t* __restrict__ nbr, int deg, Phys ph,
                                                     long long* __restrict__ bpart) {
    __shared__ long long red[4 * 4];
    const int tid = threadIdx.x;
    const long long j = blockIdx.x * 256LL + tid;
    double acc[4] = {0, 0, 0, 0};
    if (j < n) {
        const uint4 q = pin[j];
        const double sx = ph.lx * kInvTwo32, sy = ph.ly * kInvTwo32, sz = ph.lz * kInvTwo32;
        for (int b = 0; b < deg; ++b) {
            const int p = nbr[j * deg + b];
            if (p < 0) break;
            const uint4 qp = pin[p];
            const double dx = sx * fixed_delta(q.x, qp.x), dy = sy * fixed_delta(q.y, qp.y),
                         dz = sz * fixed_delta(q.z, qp.z);
            acc[0] += 0.5 * ph.bond_k * (dx * dx + dy * dy + dz * dz);
            acc[1] -= ph.bond_k * dx * dx;
            acc[2] -= ph.bond_k * dy * dy;
            acc[3] -= ph.bond_k * dz * dz;
        }
    }
    // 32.32 fixed point: the total does not depend on the order of the beads
    long long fx[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) fx[q] = llrint(acc[q] * kTwo32);
    block_sum<long long, 4>(fx, red, tid, 256);
    if (tid == 0)
        for (int q = 0; q < 4; ++q) bpart[blockIdx.x * 4 + q] = fx[q];
}

// Deterministic final sum (fixed order) of the energy partials.
__global__ void __launch_bounds__(256) k_reduce_energy(const double* __restrict__ epart, int nz,
                                                       const long long* __restrict__ bpart, int nb, Phys ph,
                                                       double n_a, double n_b, double* __restrict__ eout) {
    __shared__ double red[kEpart * 4];
    __shared__ long long bred[4 * 4];
    const int tid = threadIdx.x;
    double acc[kEpart];
    for (int q = 0; q < kEpart; ++q) acc[q] = 0.0;
    for (int i = tid; i < nz; i += 256)
        for (int q = 0; q < kEpart; ++q) acc[q] += epart[i * kEpart + q];
    long long bacc[4] = {0, 0, 0, 0};
    for (int i = tid; i < nb; i += 256)
        for (int q = 0; q < 4; ++q) bacc[q] += bpart[i * 4 + q];
    block_sum<long long, 4>(bacc, bred, tid, 256);
    block_sum<double, kEpart>(acc, red, tid, 256);
    if (tid == 0) {
        const double e_chi = ph.chi * ph.inv_n * acc[0] + ph.chi * n_a * n_b * ph.inv_n * ph.u0;
        const double e_kap = 0.5 * ph.kappa * ph.inv_n * acc[1];
        // electrostatics: E_e = (1/2) sum W_e |rho_e|^2; W_aa gets
        // (1/2) sum W_e |rho_e|^2 [1 - 2 k_a^2 (1/k^2 + a_e^2)]
        const double e_el = 0.5 * acc[5];
        double wb[3];
        for (int a = 0; a < 3; ++a) wb[a] = (double)bacc[1 + a] * kInvTwo32;
        const double e_b = (double)bacc[0] * kInvTwo32;
        eout[0] = e_b;
        eout[1] = e_chi;
        eout[2] = e_kap;
        eout[3] = e_b + e_chi + e_kap + e_el;
        for (int a = 0; a < 3; ++a) eout[4 + a] = -2.0 * ph.a2 * acc[2 + a] + wb[a] + e_el - acc[6 + a];
        eout[7] = e_el;
        // parameter gradients of the non-bonded energy at fixed positions
        eout[8] = ph.inv_n * (acc[0] + n_a * n_b * ph.u0);                       // dE/dchi
        eout[9] = 0.5 * ph.inv_n * acc[1];                                       // dE/dkappa
        eout[10] = ph.sampled ? __builtin_nan("") : -2.0 * sqrt(ph.a2) * (acc[2] + acc[3] + acc[4]);  // dE/da
    }
}

__global__ void __launch_bounds__(256) k_stream_copy(uint4* __restrict__ dst, const uint4* __restrict__ src,
                                                     long long n16) {
    const long long stride = (long long)gridDim.x * 256;
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
}

size_t plane_lds_bytes(const Launch& L) {
    const size_t c = L.precision == 0 ? sizeof(float2) : sizeof(double2);
    return c * ((size_t)L.d.npg * (size_t)(2 * L.d.hxp) + (size_t)L.d.ntw());
}

size_t z_lds_bytes(const Launch& L) {
    const size_t c = L.precision == 0 ? sizeof(float2) : sizeof(double2);
    return c * (4 * (size_t)L.d.mz * (size_t)(L.z_cols | 1) + (size_t)L.d.ntw()) +
           sizeof(ZPlane) * (size_t)L.d.mz + sizeof(ZColumn) * (size_t)L.z_cols;
}

template <typename T, int EO, bool EL> static void z_te(const Launch& L, DeviceState& S, int want_energy) {
    hipLaunchKernelGGL((k_z_kmul<T, kZBlock, EO, EL>), dim3(L.n_zblocks), dim3(kZBlock), z_lds_bytes(L), L.stream,
                       (const cplx<T>*)S.spec, (cplx<T>*)S.zout, L.d, L.pz, (const cplx<T>*)S.tw, L.ph, L.z_cols,
                       S.epart, want_energy, S.noise_step && !L.force_ad ? S.noise_part : nullptr, S.n, S.qshift,
                       S.qshift_next, S.utab, S.vtab, L.force_ad ? 2 : 4, (const RepDesc*)nullptr, (const uint32_t*)nullptr, 0);
}

template <typename T, int EO> static void z_t(const Launch& L, DeviceState& S, int want_energy) {
    if (L.ph.elec) z_te<T, EO, true>(L, S, want_energy);
    else z_te<T, EO, false>(L, S, want_energy);
}

hipError_t launch_z_kmul(const Launch& L, DeviceState& S, bool energy_only, bool with_energy) {
    const int we = (energy_only || with_energy) ? 1 : 0;
    if (L.precision == 0) {
        if (energy_only) z_t<float, 1>(L, S, 1);
        else z_t<float, 0>(L, S, we);
    } else {
        if (energy_only) z_t<double, 1>(L, S, 1);
        else z_t<double, 0>(L, S, we);
    }
    return hipGetLastError();
}

template <typename T, int P, int MODE>
static void update_p(const Launch& L, DeviceState& S, uint64_t step, void* out, int out_dtype, unsigned parts,
                     double out_sign) {
    // Euler-Maruyama steps: kStepBeads beads per thread; GJF steps (two draws
    // per bead, the velocities) and forces only: one; at least one block
    constexpr int NB = MODE == 0 ? kStepBeads : 1;
    const unsigned g = blocks_for(S.n > 0 ? S.n : 1, 256 * NB);
    hipLaunchKernelGGL((k_update<T, P, MODE, false, NB>), dim3(g), dim3(256), 0, L.stream, S.pos, S.pos_tmp,
                       (const T*)S.fbond, (const T*)S.fpart, S.qshift_next, S.n, L.d, L.ph, step, out, out_dtype,
                       parts, out_sign, S.kr, S.counts, S.flag, S.qshift, (const T*)S.vel, (T*)S.vel_tmp,
                       (const RepDesc*)nullptr, (const uint32_t*)nullptr, 0);
}

template <typename T, int MODE>
static void update_t(const Launch& L, DeviceState& S, uint64_t step, void* out, int od, unsigned parts, double sg) {
    switch (L.order) {
        case 1: update_p<T, 1, MODE>(L, S, step, out, od, parts, sg); break;
        case 2: update_p<T, 2, MODE>(L, S, step, out, od, parts, sg); break;
        case 3: update_p<T, 3, MODE>(L, S, step, out, od, parts, sg); break;
        case 4: update_p<T, 4, MODE>(L, S, step, out, od, parts, sg); break;
        case 5: update_p<T, 5, MODE>(L, S, step, out, od, parts, sg); break;
        case 6: update_p<T, 6, MODE>(L, S, step, out, od, parts, sg); break;
        default: update_p<T, 7, MODE>(L, S, step, out, od, parts, sg); break;
    }
}

hipError_t launch_update(const Launch& L, DeviceState& S, int mode, uint64_t step, void* out, int out_dtype,
                         unsigned parts, double out_sign) {
    if (mode == 0 && L.force_ad)
        hipLaunchKernelGGL(k_form_shift, dim3(1), dim3(kShiftBlock), 0, L.stream, S.noise_part, S.fsum_part, 2 * L.d.mz,
                           S.n, L.ph, S.qshift, S.qshift_next);
    const bool gjf = mode == 0 && L.ph.gjf;
    if (L.precision == 0) {
        if (gjf) update_t<float, 2>(L, S, step, out, out_dtype, parts, out_sign);
        else if (mode == 0) update_t<float, 0>(L, S, step, out, out_dtype, parts, out_sign);
        else update_t<float, 1>(L, S, step, out, out_dtype, parts, out_sign);
    } else {
        if (gjf) update_t<double, 2>(L, S, step, out, out_dtype, parts, out_sign);
        else if (mode == 0) update_t<double, 0>(L, S, step, out, out_dtype, parts, out_sign);
        else update_t<double, 1>(L, S, step, out, out_dtype, parts, out_sign);
    }
    return hipGetLastError();
}

hipError_t launch_bin_scan(const Launch& L, DeviceState& S) {
    const unsigned ntiles = (unsigned)((S.nbins + kScanBins - 1) / kScanBins);
    hipLaunchKernelGGL(k_bin_scan<false>, dim3(ntiles), dim3(256), 0, L.stream, S.counts, S.bin_start, S.nbins,
                       S.scan_status, S.scan_status + ntiles, S.flag, (const RepDesc*)nullptr, (const uint32_t*)nullptr);
    return hipGetLastError();
}

template <typename T, int NB, int DEG>
static void scatter_t(const Launch& L, DeviceState& S, const int32_t* nbr_src, long long* np, uint64_t ns) {
    hipLaunchKernelGGL((k_scatter<T, false, NB, DEG>), dim3(blocks_for(S.n, 256 * NB)), dim3(256), 0, L.stream,
                       S.pos_tmp, S.kr, S.bin_start, nbr_src, S.pos, S.nbr_old, (T*)S.fbond, S.n, S.deg, L.ph,
                       (const T*)S.vel_tmp, (T*)S.vel, (const RepDesc*)nullptr, (const uint32_t*)nullptr, 0, S.grec,
                       S.qshift, L.d, L.order, np, ns);
}

template <typename T>
static void scatter_deg(const Launch& L, DeviceState& S, const int32_t* nbr_src, long long* np, uint64_t ns) {
    // partner tables up to four columns wide are held in registers; GJF (two
    // draws per bead for the noise sums, the velocities) keeps one bead per thread
    if (L.ph.gjf) {
        switch (S.deg) {
            case 1: scatter_t<T, 1, 1>(L, S, nbr_src, np, ns); break;
            case 2: scatter_t<T, 1, 2>(L, S, nbr_src, np, ns); break;
            case 3: scatter_t<T, 1, 3>(L, S, nbr_src, np, ns); break;
            case 4: scatter_t<T, 1, 4>(L, S, nbr_src, np, ns); break;
            default: scatter_t<T, 1, 0>(L, S, nbr_src, np, ns); break;
        }
        return;
    }
    switch (S.deg) {
        case 1: scatter_t<T, kStepBeads, 1>(L, S, nbr_src, np, ns); break;
        case 2: scatter_t<T, kStepBeads, 2>(L, S, nbr_src, np, ns); break;
        case 3: scatter_t<T, kStepBeads, 3>(L, S, nbr_src, np, ns); break;
        case 4: scatter_t<T, kStepBeads, 4>(L, S, nbr_src, np, ns); break;
        default: scatter_t<T, 1, 0>(L, S, nbr_src, np, ns); break;
    }
}

hipError_t launch_scatter(const Launch& L, DeviceState& S, const int32_t* nbr_src, int64_t noise_step) {
    if (S.n == 0) return hipSuccess;
    long long* np = noise_step >= 0 ? S.noise_part : nullptr;
    const uint64_t ns = noise_step >= 0 ? (uint64_t)noise_step : 0u;
    if (L.precision == 0) scatter_deg<float>(L, S, nbr_src, np, ns);
    else scatter_deg<double>(L, S, nbr_src, np, ns);
    return hipGetLastError();
}

hipError_t launch_noise_sum(const Launch& L, DeviceState& S, uint64_t step) {
    const unsigned g = blocks_for(S.n > 0 ? S.n : 1, 256);
    if (L.precision == 0)
        hipLaunchKernelGGL((k_noise_sum<float, false>), dim3(g), dim3(256), 0, L.stream, S.pos, S.n, L.ph, step,
                           S.noise_part, (const RepDesc*)nullptr, (const uint32_t*)nullptr);
    else
        hipLaunchKernelGGL((k_noise_sum<double, false>), dim3(g), dim3(256), 0, L.stream, S.pos, S.n, L.ph, step,
                           S.noise_part, (const RepDesc*)nullptr, (const uint32_t*)nullptr);
    return hipGetLastError();
}

hipError_t launch_bond_energy(const Launch& L, DeviceState& S) {
    hipLaunchKernelGGL(k_bond_energy, dim3(L.n_bblocks), dim3(256), 0, L.stream, S.pos, S.n, S.nbr, S.deg, L.ph,
                       S.bpart);
    return hipGetLastError();
}

hipError_t launch_reduce_energy(const Launch& L, DeviceState& S) {
    hipLaunchKernelGGL(k_reduce_energy, dim3(1), dim3(256), 0, L.stream, S.epart, L.n_zblocks, S.bpart, L.n_bblocks,
                       L.ph, (double)S.n_a, (double)S.n_b, S.eout);
    return hipGetLastError();
}

hipError_t launch_place(const Launch& L, DeviceState& S, const void* xyz, int dtype) {
    const unsigned g = blocks_for(S.n > 0 ? S.n : 1, 256);
    if (dtype == 0)
        hipLaunchKernelGGL(k_place<float>, dim3(g), dim3(256), 0, L.stream, (const float*)xyz, S.types_abi, S.pos_tmp,
                           S.kr, S.counts, S.qshift, S.n, L.d, L.order, S.flag);
    else
        hipLaunchKernelGGL(k_place<double>, dim3(g), dim3(256), 0, L.stream, (const double*)xyz, S.types_abi,
                           S.pos_tmp, S.kr, S.counts, S.qshift, S.n, L.d, L.order, S.flag);
    return hipGetLastError();
}

template <typename T>
static void velocities_t(const Launch& L, DeviceState& S, int op, void* v, int dtype) {
    const unsigned g = blocks_for(S.n, 256);
    T* vel = (T*)S.vel;
    T* vt = (T*)S.vel_tmp;
    if (op == 2)
        hipLaunchKernelGGL((k_velocities<T, T, 2>), dim3(g), dim3(256), 0, L.stream, S.pos, vel, vt, (T*)nullptr, S.n);
    else if (dtype == 0) {
        if (op == 0)
            hipLaunchKernelGGL((k_velocities<T, float, 0>), dim3(g), dim3(256), 0, L.stream, S.pos, vel, vt, (float*)v,
                               S.n);
        else
            hipLaunchKernelGGL((k_velocities<T, float, 1>), dim3(g), dim3(256), 0, L.stream, S.pos, vel, vt, (float*)v,
                               S.n);
    } else {
        if (op == 0)
            hipLaunchKernelGGL((k_velocities<T, double, 0>), dim3(g), dim3(256), 0, L.stream, S.pos, vel, vt,
                               (double*)v, S.n);
        else
            hipLaunchKernelGGL((k_velocities<T, double, 1>), dim3(g), dim3(256), 0, L.stream, S.pos, vel, vt,
                               (double*)v, S.n);
    }
}

hipError_t launch_velocities(const Launch& L, DeviceState& S, int op, void* v, int dtype) {
    if (S.n == 0 || !S.vel) return hipSuccess;
    if (L.precision == 0) velocities_t<float>(L, S, op, v, dtype);
    else velocities_t<double>(L, S, op, v, dtype);
    return hipGetLastError();
}

template <typename T>
static void bead_vectors_t(const Launch& L, DeviceState& S, T* sorted, int op, void* v, int dtype) {
    const unsigned g = blocks_for(S.n, 256);
    if (dtype == 0) {
        if (op == 0)
            hipLaunchKernelGGL((k_velocities<T, float, 0>), dim3(g), dim3(256), 0, L.stream, S.pos, sorted, (T*)nullptr,
                               (float*)v, S.n);
        else
            hipLaunchKernelGGL((k_velocities<T, float, 1>), dim3(g), dim3(256), 0, L.stream, S.pos, sorted, (T*)nullptr,
                               (float*)v, S.n);
    } else {
        if (op == 0)
            hipLaunchKernelGGL((k_velocities<T, double, 0>), dim3(g), dim3(256), 0, L.stream, S.pos, sorted,
                               (T*)nullptr, (double*)v, S.n);
        else
            hipLaunchKernelGGL((k_velocities<T, double, 1>), dim3(g), dim3(256), 0, L.stream, S.pos, sorted,
                               (T*)nullptr, (double*)v, S.n);
    }
}

hipError_t launch_bead_vectors(const Launch& L, DeviceState& S, void* sorted, int op, void* v, int dtype) {
    if (S.n == 0) return hipSuccess;
    if (L.precision == 0) bead_vectors_t<float>(L, S, (float*)sorted, op, v, dtype);
    else bead_vectors_t<double>(L, S, (double*)sorted, op, v, dtype);
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

// The plane kernels of one context: the same block sizes and order as the launchers above pick.

template <typename T> static hipError_t attr_z(size_t lds) {
    const void* fns[4] = {(const void*)k_z_kmul<T, kZBlock, 0, false>, (const void*)k_z_kmul<T, kZBlock, 1, false>,
                          (const void*)k_z_kmul<T, kZBlock, 0, true>, (const void*)k_z_kmul<T, kZBlock, 1, true>};
    for (const void* f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t configure_kernel_attributes(const Launch& L) {
    const size_t lp = plane_lds_bytes(L), lz = z_lds_bytes(L);
    hipError_t e = hipSuccess;
    if (L.precision == 0) {
        e = configure_plane_attributes(L, lp);
        if (e == hipSuccess) e = configure_second_attributes(L, lp);
        if (e == hipSuccess) e = attr_z<float>(lz);
    } else {
        e = configure_plane_attributes(L, lp);
        if (e == hipSuccess) e = configure_second_attributes(L, lp);
        if (e == hipSuccess) e = attr_z<double>(lz);
    }
    return e;
}

}  // namespace tild

// Launchers of the batched step: one launch per kernel for every member of a
// batch of contexts.
#include "tild_device.h"

namespace tild {

// ------------------------------------------------------------ batched step

template <typename T, int PB>
static void batch_step_t(const Launch& L, const BatchMaps& B, int s, size_t lp, size_t lz) {
    const RepDesc* R = B.reps;
    const uint64_t so = (uint64_t)s;
    const int par = s & 1;
    with_order(L.order, [&](auto Pc) {
        constexpr int P = decltype(Pc)::value;
        // members of large planes, then those of small planes (fewer threads, their own LDS size)
        const int nbig_plane = B.n_plane - B.n_plane_small, nbig_c2r = B.n_c2r - B.n_c2r_small;
        if (nbig_plane > 0)
            hipLaunchKernelGGL((k_spread_xy<T, PB, P, true>), dim3(nbig_plane), dim3(PB), lp, L.stream,
                               (const uint4*)nullptr, (const uint32_t*)nullptr, (const uint32_t*)nullptr,
                               (cplx<T>*)nullptr, L.d, L.px, L.py, (const cplx<T>*)nullptr, L.ph, (uint32_t*)nullptr,
                               R, B.plane, par, (const T*)nullptr, (T*)nullptr, 0);
        if (B.n_plane_small > 0)
            hipLaunchKernelGGL((k_spread_xy<T, kSmallPlaneBlock, P, true>), dim3(B.n_plane_small),
                               dim3(kSmallPlaneBlock), B.lds_small, L.stream, (const uint4*)nullptr,
                               (const uint32_t*)nullptr, (const uint32_t*)nullptr, (cplx<T>*)nullptr, L.d, L.px, L.py,
                               (const cplx<T>*)nullptr, L.ph, (uint32_t*)nullptr, R, B.plane + nbig_plane, par,
                               (const T*)nullptr, (T*)nullptr, 0);
        if (L.ph.elec)
            hipLaunchKernelGGL((k_z_kmul<T, kZBlock, 0, true, true>), dim3(B.n_zcol), dim3(kZBlock), lz, L.stream,
                               (const cplx<T>*)nullptr, (cplx<T>*)nullptr, L.d, L.pz, (const cplx<T>*)nullptr, L.ph, 1,
                               (double*)nullptr, 0, (const long long*)nullptr, 0LL, (const uint32_t*)nullptr,
                               (uint32_t*)nullptr, (const double*)nullptr, (const double*)nullptr, 4, R, B.zcol, par);
        else
            hipLaunchKernelGGL((k_z_kmul<T, kZBlock, 0, false, true>), dim3(B.n_zcol), dim3(kZBlock), lz, L.stream,
                               (const cplx<T>*)nullptr, (cplx<T>*)nullptr, L.d, L.pz, (const cplx<T>*)nullptr, L.ph, 1,
                               (double*)nullptr, 0, (const long long*)nullptr, 0LL, (const uint32_t*)nullptr,
                               (uint32_t*)nullptr, (const double*)nullptr, (const double*)nullptr, 4, R, B.zcol, par);
        if (nbig_c2r > 0)
            hipLaunchKernelGGL((k_xy_c2r<T, PB, P, false, true>), dim3(nbig_c2r), dim3(PB), lp, L.stream,
                               (const cplx<T>*)nullptr, (T*)nullptr, L.d, L.px, L.py, (const cplx<T>*)nullptr, L.ph,
                               (const uint4*)nullptr, (const uint32_t*)nullptr, (const uint32_t*)nullptr, 0LL,
                               (long long*)nullptr, R, B.c2r, par, (const T*)nullptr, (const T*)nullptr, 0,
                               (T*)nullptr, 0);
        if (B.n_c2r_small > 0)
            hipLaunchKernelGGL((k_xy_c2r<T, kSmallPlaneBlock, P, false, true>), dim3(B.n_c2r_small),
                               dim3(kSmallPlaneBlock), B.lds_small, L.stream, (const cplx<T>*)nullptr, (T*)nullptr,
                               L.d, L.px, L.py, (const cplx<T>*)nullptr, L.ph, (const uint4*)nullptr,
                               (const uint32_t*)nullptr, (const uint32_t*)nullptr, 0LL, (long long*)nullptr, R,
                               B.c2r + nbig_c2r, par, (const T*)nullptr, (const T*)nullptr, 0, (T*)nullptr, 0);
        hipLaunchKernelGGL((k_update<T, P, 0, true>), dim3(B.n_bead), dim3(256), 0, L.stream, (const uint4*)nullptr,
                           (uint4*)nullptr, (const T*)nullptr, (const T*)nullptr, (const uint32_t*)nullptr, 0LL, L.d,
                           L.ph, so, (void*)nullptr, 0, 0u, 1.0, (uint2*)nullptr, (uint32_t*)nullptr,
                           (uint32_t*)nullptr, (const uint32_t*)nullptr, (const T*)nullptr, (T*)nullptr, R, B.bead,
                           par);
    });
    hipLaunchKernelGGL(k_bin_scan<true>, dim3(B.n_tile), dim3(256), 0, L.stream, (uint32_t*)nullptr,
                       (uint32_t*)nullptr, 0, (unsigned long long*)nullptr, B.ticket, (uint32_t*)nullptr, R, B.tile);
    // partners in registers where every member's partner table has the same width (1..4)
    auto scatter = [&](auto Dc) {
        constexpr int DEG = decltype(Dc)::value;
        hipLaunchKernelGGL((k_scatter<T, true, 1, DEG>), dim3(B.n_bead), dim3(256), 0, L.stream,
                           (const uint4*)nullptr, (const uint2*)nullptr, (const uint32_t*)nullptr,
                           (const int32_t*)nullptr, (uint4*)nullptr, (int32_t*)nullptr, (T*)nullptr, 0LL, 0, L.ph,
                           (const T*)nullptr, (T*)nullptr, R, B.bead, par, (uint4*)nullptr, (const uint32_t*)nullptr,
                           L.d, L.order, (long long*)nullptr, so + 1);
    };
    switch (B.deg) {
        case 1: scatter(std::integral_constant<int, 1>{}); break;
        case 2: scatter(std::integral_constant<int, 2>{}); break;
        case 3: scatter(std::integral_constant<int, 3>{}); break;
        case 4: scatter(std::integral_constant<int, 4>{}); break;
        default: scatter(std::integral_constant<int, 0>{}); break;
    }
}

hipError_t launch_batch_noise(const Launch& L, const BatchMaps& B) {
    if (L.precision == 0)
        hipLaunchKernelGGL((k_noise_sum<float, true>), dim3(B.n_bead), dim3(256), 0, L.stream, (const uint4*)nullptr, 0LL,
                           L.ph, (uint64_t)0, (long long*)nullptr, B.reps, B.bead);
    else
        hipLaunchKernelGGL((k_noise_sum<double, true>), dim3(B.n_bead), dim3(256), 0, L.stream, (const uint4*)nullptr,
                           0LL, L.ph, (uint64_t)0, (long long*)nullptr, B.reps, B.bead);
    return hipGetLastError();
}

hipError_t launch_batch_step(const Launch& L, const BatchMaps& B, int s, size_t lds_plane, size_t lds_z) {
    if (L.precision == 0) {
        if (B.plane_block == 256) batch_step_t<float, 256>(L, B, s, lds_plane, lds_z);
        else batch_step_t<float, 512>(L, B, s, lds_plane, lds_z);
    } else {
        if (B.plane_block == 256) batch_step_t<double, 256>(L, B, s, lds_plane, lds_z);
        else batch_step_t<double, 512>(L, B, s, lds_plane, lds_z);
    }
    return hipGetLastError();
}

template <typename T> static hipError_t attr_batch(const Launch& L, size_t lp, size_t lz) {
    hipError_t e = hipSuccess;
    auto set = [&](const void* f, size_t b) {
        if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)b);
    };
    with_order(L.order, [&](auto Pc) {
        constexpr int P = decltype(Pc)::value;
        set((const void*)k_spread_xy<T, 256, P, true>, lp);
        set((const void*)k_xy_c2r<T, 256, P, false, true>, lp);
        set((const void*)k_spread_xy<T, 512, P, true>, lp);
        set((const void*)k_xy_c2r<T, 512, P, false, true>, lp);
    });
    set((const void*)k_z_kmul<T, kZBlock, 0, false, true>, lz);
    set((const void*)k_z_kmul<T, kZBlock, 0, true, true>, lz);
    return e;
}

hipError_t configure_batch_attributes(const Launch& L, size_t lds_plane, size_t lds_z) {
    return L.precision == 0 ? attr_batch<float>(L, lds_plane, lds_z) : attr_batch<double>(L, lds_plane, lds_z);
}

}  // namespace tild

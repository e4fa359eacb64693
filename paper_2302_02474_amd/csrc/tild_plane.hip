// Launchers of the plane kernels: the fused spread and forward xy pass and the
// inverse xy pass with the interpolation.
#include "tild_device.h"

namespace tild {

template <typename T, int B> static void spread_xy_b(const Launch& L, DeviceState& S) {
    with_order(L.order, [&](auto Pc) {
        hipLaunchKernelGGL((k_spread_xy<T, B, decltype(Pc)::value>), dim3(L.d.mz, 2), dim3(B), plane_lds_bytes(L),
                           L.stream, bead_src(L, S), S.bin_start, S.qshift, (cplx<T>*)S.spec, L.d, L.px, L.py,
                           (const cplx<T>*)S.tw, L.ph, S.flag, S.noise_step ? 1 : 0, (uint64_t)S.step, S.noise_part,
                           (const RepDesc*)nullptr, (const uint32_t*)nullptr, 0, (const T*)nullptr, (T*)nullptr, 0);
    });
}
template <typename T, int B> static void xy_c2r_b(const Launch& L, DeviceState& S, bool ad) {
    with_order(L.order, [&](auto Pc) {
        constexpr int P = decltype(Pc)::value;
        if (ad)
            hipLaunchKernelGGL((k_xy_c2r<T, B, P, true>), dim3(L.d.mz, 2), dim3(B), plane_lds_bytes(L), L.stream,
                               (const cplx<T>*)S.zout, (T*)S.fpart, L.d, L.px, L.py, (const cplx<T>*)S.tw, L.ph,
                               bead_src(L, S), S.bin_start, S.qshift, S.n, S.fsum_part, (const RepDesc*)nullptr,
                               (const uint32_t*)nullptr, 0, (const T*)nullptr, (const T*)nullptr, 0, (T*)nullptr);
        else
            hipLaunchKernelGGL((k_xy_c2r<T, B, P, false>), dim3(L.d.mz, 2, 3), dim3(B), plane_lds_bytes(L),
                               L.stream, (const cplx<T>*)S.zout, (T*)S.fpart, L.d, L.px, L.py, (const cplx<T>*)S.tw,
                               L.ph, bead_src(L, S), S.bin_start, S.qshift, S.n, S.fsum_part, (const RepDesc*)nullptr,
                               (const uint32_t*)nullptr, 0, (const T*)nullptr, (const T*)nullptr, 0, (T*)nullptr);
    });
}

hipError_t launch_spread_xy(const Launch& L, DeviceState& S) {
    if (L.precision == 0) {
        if (L.spread_block == 256) spread_xy_b<float, 256>(L, S);
        else if (L.spread_block == 512) spread_xy_b<float, 512>(L, S);
        else spread_xy_b<float, 1024>(L, S);
    } else {
        if (L.spread_block == 256) spread_xy_b<double, 256>(L, S);
        else spread_xy_b<double, 512>(L, S);
    }
    return hipGetLastError();
}

hipError_t launch_xy_c2r(const Launch& L, DeviceState& S, int route) {
    const bool ad = route < 0 ? L.force_ad != 0 : route == 1;
    if (L.precision == 0) {
        if (L.plane_block == 256) xy_c2r_b<float, 256>(L, S, ad);
        else xy_c2r_b<float, 512>(L, S, ad);
    } else {
        if (L.plane_block == 256) xy_c2r_b<double, 256>(L, S, ad);
        else xy_c2r_b<double, 512>(L, S, ad);
    }
    return hipGetLastError();
}

template <typename T> static hipError_t attr_plane(const Launch& L, size_t lds) {
    hipError_t e = hipSuccess;
    auto set = [&](const void* f) {
        if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    };
    with_order(L.order, [&](auto Pc) {
        constexpr int P = decltype(Pc)::value;
        if (L.spread_block == 256) set((const void*)k_spread_xy<T, 256, P>);
        else if constexpr (sizeof(T) == 8) set((const void*)k_spread_xy<T, 512, P>);
        else if (L.spread_block == 512) set((const void*)k_spread_xy<T, 512, P>);
        else set((const void*)k_spread_xy<T, 1024, P>);
        if (L.plane_block == 256) {
            set((const void*)k_xy_c2r<T, 256, P, false>);
            set((const void*)k_xy_c2r<T, 256, P, true>);
        } else {
            set((const void*)k_xy_c2r<T, 512, P, false>);
            set((const void*)k_xy_c2r<T, 512, P, true>);
        }
    });
    return e;
}

hipError_t configure_plane_attributes(const Launch& L, size_t lds) {
    return L.precision == 0 ? attr_plane<float>(L, lds) : attr_plane<double>(L, lds);
}

}  // namespace tild

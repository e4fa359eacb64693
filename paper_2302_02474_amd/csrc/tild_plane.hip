// Launchers of the plane kernels: the fused spread and forward xy pass and the
// inverse xy pass with the interpolation.
//
// Compiled twice, for the single-precision kernels (this file; it also holds
// the precision dispatch) and for the double-precision ones
// (tild_plane_f64.hip, TILD_PART_F64), so the two halves build side by side.
#include "tild_device.h"

namespace tild {

hipError_t plane_spread_f64(const Launch& L, DeviceState& S);
hipError_t plane_c2r_f64(const Launch& L, DeviceState& S, bool ad);
hipError_t plane_attr_f64(const Launch& L, size_t lds);

template <typename T, int B> static void spread_xy_b(const Launch& L, DeviceState& S) {
    with_order(L.order, [&](auto Pc) {
        hipLaunchKernelGGL((k_spread_xy<T, B, decltype(Pc)::value>), dim3(L.d.mz, 2), dim3(B), plane_lds_bytes(L),
                           L.stream, bead_src(L, S), S.bin_start, S.qshift, (cplx<T>*)S.spec, L.d, L.px, L.py,
                           (const cplx<T>*)S.tw, L.ph, S.flag, (const RepDesc*)nullptr, (const uint32_t*)nullptr, 0,
                           (const T*)nullptr, (T*)nullptr, 0);
    });
}
template <typename T, int B> static void xy_c2r_b(const Launch& L, DeviceState& S, bool ad) {
    const size_t lds = plane_lds_bytes(L);
    with_order(L.order, [&](auto Pc) {
        constexpr int P = decltype(Pc)::value;
        if (ad) {
            hipLaunchKernelGGL((k_xy_c2r<T, B, P, true>), dim3(L.d.mz, 2), dim3(B), lds, L.stream,
                               (const cplx<T>*)S.zout, (T*)S.fpart, L.d, L.px, L.py, (const cplx<T>*)S.tw, L.ph,
                               bead_src(L, S), S.bin_start, S.qshift, S.n, S.fsum_part, (const RepDesc*)nullptr,
                               (const uint32_t*)nullptr, 0, (const T*)nullptr, (const T*)nullptr, 0, (T*)nullptr, 0);
            return;
        }
        hipLaunchKernelGGL((k_xy_c2r<T, B, P, false>), dim3(6 * L.d.mz), dim3(B), lds, L.stream,
                           (const cplx<T>*)S.zout, (T*)S.fpart, L.d, L.px, L.py, (const cplx<T>*)S.tw, L.ph,
                           bead_src(L, S), S.bin_start, S.qshift, S.n, S.fsum_part, (const RepDesc*)nullptr,
                           (const uint32_t*)nullptr, 0, (const T*)nullptr, (const T*)nullptr, 0, (T*)nullptr, 0);
    });
}

#ifndef TILD_PART_F64
hipError_t launch_spread_xy(const Launch& L, DeviceState& S) {
    if (L.precision != 0) return plane_spread_f64(L, S);
    if (L.spread_block == 256) spread_xy_b<float, 256>(L, S);
    else if (L.spread_block == 512) spread_xy_b<float, 512>(L, S);
    else spread_xy_b<float, 1024>(L, S);
    return hipGetLastError();
}

hipError_t launch_xy_c2r(const Launch& L, DeviceState& S, int route) {
    const bool ad = route < 0 ? L.force_ad != 0 : route == 1;
    if (L.precision != 0) return plane_c2r_f64(L, S, ad);
    if (L.plane_block == 256) xy_c2r_b<float, 256>(L, S, ad);
    else xy_c2r_b<float, 512>(L, S, ad);
    return hipGetLastError();
}
#else
hipError_t plane_spread_f64(const Launch& L, DeviceState& S) {
    if (L.spread_block == 256) spread_xy_b<double, 256>(L, S);
    else spread_xy_b<double, 512>(L, S);
    return hipGetLastError();
}

hipError_t plane_c2r_f64(const Launch& L, DeviceState& S, bool ad) {
    if (L.plane_block == 256) xy_c2r_b<double, 256>(L, S, ad);
    else xy_c2r_b<double, 512>(L, S, ad);
    return hipGetLastError();
}
#endif

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

#ifndef TILD_PART_F64
hipError_t configure_plane_attributes(const Launch& L, size_t lds) {
    return L.precision == 0 ? attr_plane<float>(L, lds) : plane_attr_f64(L, lds);
}
#else
hipError_t plane_attr_f64(const Launch& L, size_t lds) { return attr_plane<double>(L, lds); }
#endif

}  // namespace tild

// Launchers of the plane kernels' other modes: mesh counts, forces of a given
// field, and Hessian-vector products (directional spread, second-derivative
// interpolation).
//
// Compiled twice, for the single-precision kernels (this file; it also holds
// the precision dispatch) and for the double-precision ones
// (tild_second_f64.hip, TILD_PART_F64), so the two halves build side by side.
#include "tild_device.h"

namespace tild {

// the double-precision halves (tild_second_f64.hip)
void second_counts_f64(const Launch& L, DeviceState& S, void* out);
void second_field_f64(const Launch& L, DeviceState& S, const void* field);
hipError_t second_hvp_f64(const Launch& L, DeviceState& S, const void* v, void* out, int dtype);
hipError_t second_hvp_tail_f64(const Launch& L, DeviceState& S, void* out, int dtype);
hipError_t second_vjp_f64(const Launch& L, DeviceState& S, void* out, int dtype);
hipError_t second_attr_f64(const Launch& L, size_t lds);

template <typename T, int B>
static hipError_t hvp_b(const Launch& L, DeviceState& S, const void* v, void* out, int dtype) {
    const hipError_t e = launch_bead_vectors(L, S, S.vdir, 0, const_cast<void*>(v), dtype);
    if (e != hipSuccess) return e;
    const unsigned gb = blocks_for(S.n, 256);
    with_order(L.order, [&](auto Pc) {
        constexpr int P = decltype(Pc)::value;
        if constexpr (P >= 3) {
            // second-derivative terms against the potential planes of the counts
            hipLaunchKernelGGL((k_xy_c2r<T, B, P, true, false, true>), dim3(L.d.mz, 2), dim3(B), plane_lds_bytes(L),
                               L.stream, (const cplx<T>*)S.zout, (T*)S.fpart, L.d, L.px, L.py, (const cplx<T>*)S.tw,
                               L.ph, bead_src(L, S), S.bin_start, S.qshift, S.n, S.fsum_part, (const RepDesc*)nullptr,
                               (const uint32_t*)nullptr, 0, (const T*)S.vdir, (const T*)nullptr, 0, (T*)nullptr, 0);
            hipLaunchKernelGGL((k_hvp_accum<T, P>), dim3(gb), dim3(256), 0, L.stream, (const T*)S.fpart, S.n,
                               (const T*)S.vdir, S.nbr, S.deg, L.ph.bond_k, (T*)S.hacc, 1, (T)1, (T)1);
            // the field of the directional counts, gathered with the weight gradients
            hipLaunchKernelGGL((k_spread_xy<T, B, P, false, true>), dim3(L.d.mz, 2), dim3(B), plane_lds_bytes(L),
                               L.stream, bead_src(L, S), S.bin_start, S.qshift, (cplx<T>*)S.spec, L.d, L.px, L.py,
                               (const cplx<T>*)S.tw, L.ph, S.flag,
                               (const RepDesc*)nullptr, (const uint32_t*)nullptr, 0, (const T*)S.vdir, (T*)nullptr, 0);
        }
    });
    return hipGetLastError();
}

template <typename T, int B> static hipError_t hvp_tail(const Launch& L, DeviceState& S, void* out, int dtype) {
    const unsigned gb = blocks_for(S.n, 256);
    with_order(L.order, [&](auto Pc) {
        constexpr int P = decltype(Pc)::value;
        if constexpr (P >= 3) {
            hipLaunchKernelGGL((k_xy_c2r<T, B, P, true>), dim3(L.d.mz, 2), dim3(B), plane_lds_bytes(L), L.stream,
                               (const cplx<T>*)S.zout, (T*)S.fpart, L.d, L.px, L.py, (const cplx<T>*)S.tw, L.ph,
                               bead_src(L, S), S.bin_start, S.qshift, S.n, S.fsum_part, (const RepDesc*)nullptr,
                               (const uint32_t*)nullptr, 0, (const T*)nullptr, (const T*)nullptr, 0, (T*)nullptr, 0);
            // those partials are -sum grad W delta phi
            hipLaunchKernelGGL((k_hvp_accum<T, P>), dim3(gb), dim3(256), 0, L.stream, (const T*)S.fpart, S.n,
                               (const T*)S.vdir, S.nbr, S.deg, L.ph.bond_k, (T*)S.hacc, 0, (T)-1, (T)1);
        }
    });
    const hipError_t e = hipGetLastError();
    return e != hipSuccess ? e : launch_bead_vectors(L, S, S.hacc, 1, out, dtype);
}

template <typename T, int B> static void counts_b(const Launch& L, DeviceState& S, void* out) {
    with_order(L.order, [&](auto Pc) {
        constexpr int P = decltype(Pc)::value;
        hipLaunchKernelGGL((k_spread_xy<T, B, P, false, false, true>), dim3(L.d.mz, 2), dim3(B), plane_lds_bytes(L),
                           L.stream, bead_src(L, S), S.bin_start, S.qshift, (cplx<T>*)S.spec, L.d, L.px, L.py,
                           (const cplx<T>*)S.tw, L.ph, S.flag, (const RepDesc*)nullptr,
                           (const uint32_t*)nullptr, 0, (const T*)nullptr, (T*)out, 0);
    });
}

#ifndef TILD_PART_F64
hipError_t launch_counts(const Launch& L, DeviceState& S, void* out) {
    if (L.precision != 0) second_counts_f64(L, S, out);
    else if (L.plane_block == 256) counts_b<float, 256>(L, S, out);
    else counts_b<float, 512>(L, S, out);
    return hipGetLastError();
}
#else
void second_counts_f64(const Launch& L, DeviceState& S, void* out) {
    if (L.plane_block == 256) counts_b<double, 256>(L, S, out);
    else counts_b<double, 512>(L, S, out);
}
#endif

template <typename T, int B> static void field_b(const Launch& L, DeviceState& S, const void* field) {
    with_order(L.order, [&](auto Pc) {
        constexpr int P = decltype(Pc)::value;
        if constexpr (P >= 2)
            hipLaunchKernelGGL((k_xy_c2r<T, B, P, true, false, false, true>), dim3(L.d.mz, 2), dim3(B),
                               plane_lds_bytes(L), L.stream, (const cplx<T>*)S.zout, (T*)S.fpart, L.d, L.px, L.py,
                               (const cplx<T>*)S.tw, L.ph, bead_src(L, S), S.bin_start, S.qshift, S.n, S.fsum_part,
                               (const RepDesc*)nullptr, (const uint32_t*)nullptr, 0, (const T*)nullptr,
                               (const T*)field, 0, (T*)nullptr, 0);
    });
}

#ifndef TILD_PART_F64
hipError_t launch_field_forces(const Launch& L, DeviceState& S, const void* field, void* out, int dtype) {
    if (L.order < 2) return hipErrorInvalidValue;
    if (L.precision != 0) second_field_f64(L, S, field);
    else if (L.plane_block == 256) field_b<float, 256>(L, S, field);
    else field_b<float, 512>(L, S, field);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_update(L, S, 1, 0, out, dtype, 1u);
    return e;
}

hipError_t launch_hvp(const Launch& L, DeviceState& S, const void* v, void* out, int dtype) {
    if (S.n == 0 || L.order < 3) return hipSuccess;
    // the potential planes of the counts: spread, k-space pass (noise off)
    hipError_t e = launch_spread_xy(L, S);
    if (e == hipSuccess) e = launch_z_kmul(L, S, false);
    if (e != hipSuccess) return e;
    if (L.precision != 0) e = second_hvp_f64(L, S, v, out, dtype);
    else e = L.plane_block == 256 ? hvp_b<float, 256>(L, S, v, out, dtype) : hvp_b<float, 512>(L, S, v, out, dtype);
    if (e == hipSuccess) e = launch_z_kmul(L, S, false);  // Phi of the directional counts
    if (e != hipSuccess) return e;
    if (L.precision != 0) return second_hvp_tail_f64(L, S, out, dtype);
    return L.plane_block == 256 ? hvp_tail<float, 256>(L, S, out, dtype) : hvp_tail<float, 512>(L, S, out, dtype);
}
#else
void second_field_f64(const Launch& L, DeviceState& S, const void* field) {
    if (L.plane_block == 256) field_b<double, 256>(L, S, field);
    else field_b<double, 512>(L, S, field);
}

hipError_t second_hvp_f64(const Launch& L, DeviceState& S, const void* v, void* out, int dtype) {
    return L.plane_block == 256 ? hvp_b<double, 256>(L, S, v, out, dtype) : hvp_b<double, 512>(L, S, v, out, dtype);
}

hipError_t second_hvp_tail_f64(const Launch& L, DeviceState& S, void* out, int dtype) {
    return L.plane_block == 256 ? hvp_tail<double, 256>(L, S, out, dtype) : hvp_tail<double, 512>(L, S, out, dtype);
}
#endif

// Transposed Jacobian of the ik-route force against lambda (held in vdir):
//   J^T lambda = -sum_a lambda_a sum_g grad W d_a phi    (local: weights move with the bead)
//               + sum_g grad W psi                        (field: psi = sum_a d_a phi of the
//                                                          lambda_a-weighted counts)
//               - H_b lambda                              (bonds),
// accumulated in hacc: acc = -H_b lambda - sum_a (local partials) - (field-gather partials),
// the field gather giving -sum_g grad W psi.
template <typename T, int B> static hipError_t vjp_b(const Launch& L, DeviceState& S, void* out, int dtype) {
    const unsigned gb = blocks_for(S.n, 256);
    const dim3 planes(L.d.mz, 2);
    const size_t lds = plane_lds_bytes(L);
    hipError_t e = hipSuccess;
    with_order(L.order, [&](auto Pc) {
        constexpr int P = decltype(Pc)::value;
        if constexpr (P >= 2) {
            // local part, one component of the gradient planes of the counts at a time
            for (int a = 0; a < 3; ++a) {
                hipLaunchKernelGGL((k_xy_c2r<T, B, P, false, false, false, false, 1>), planes, dim3(B), lds, L.stream,
                                   (const cplx<T>*)S.zout, (T*)S.fpart, L.d, L.px, L.py, (const cplx<T>*)S.tw, L.ph,
                                   bead_src(L, S), S.bin_start, S.qshift, S.n, S.fsum_part, (const RepDesc*)nullptr,
                                   (const uint32_t*)nullptr, 0, (const T*)S.vdir, (const T*)nullptr, a, (T*)nullptr, 0);
                hipLaunchKernelGGL((k_hvp_accum<T, P>), dim3(gb), dim3(256), 0, L.stream, (const T*)S.fpart, S.n,
                                   (const T*)S.vdir, S.nbr, S.deg, L.ph.bond_k, (T*)S.hacc, a == 0 ? 1 : 0, (T)-1,
                                   (T)-1);
            }
            // field part: psi = sum_a d_a phi[lambda_a-weighted counts], accumulated in S.field
            for (int a = 0; a < 3 && e == hipSuccess; ++a) {
                hipLaunchKernelGGL((k_spread_xy<T, B, P, false, true, false, true>), planes, dim3(B), lds, L.stream,
                                   bead_src(L, S), S.bin_start, S.qshift, (cplx<T>*)S.spec, L.d, L.px, L.py,
                                   (const cplx<T>*)S.tw, L.ph, S.flag,
                                   (const RepDesc*)nullptr, (const uint32_t*)nullptr, 0, (const T*)S.vdir,
                                   (T*)nullptr, a);
                e = launch_z_kmul(L, S, false);
                if (e == hipSuccess)
                    hipLaunchKernelGGL((k_xy_c2r<T, B, P, false, false, false, false, 2>), planes, dim3(B), lds,
                                       L.stream, (const cplx<T>*)S.zout, (T*)S.fpart, L.d, L.px, L.py,
                                       (const cplx<T>*)S.tw, L.ph, bead_src(L, S), S.bin_start, S.qshift, S.n,
                                       S.fsum_part, (const RepDesc*)nullptr, (const uint32_t*)nullptr, 0,
                                       (const T*)nullptr, (const T*)nullptr, a, (T*)S.field, 0);
            }
            if (e == hipSuccess) {
                hipLaunchKernelGGL((k_xy_c2r<T, B, P, true, false, false, true>), planes, dim3(B), lds, L.stream,
                                   (const cplx<T>*)S.zout, (T*)S.fpart, L.d, L.px, L.py, (const cplx<T>*)S.tw, L.ph,
                                   bead_src(L, S), S.bin_start, S.qshift, S.n, S.fsum_part, (const RepDesc*)nullptr,
                                   (const uint32_t*)nullptr, 0, (const T*)nullptr, (const T*)S.field, 0,
                                   (T*)nullptr, 0);
                hipLaunchKernelGGL((k_hvp_accum<T, P>), dim3(gb), dim3(256), 0, L.stream, (const T*)S.fpart, S.n,
                                   (const T*)S.vdir, S.nbr, S.deg, L.ph.bond_k, (T*)S.hacc, 0, (T)-1, (T)-1);
            }
        }
    });
    if (e == hipSuccess) e = hipGetLastError();
    return e != hipSuccess ? e : launch_bead_vectors(L, S, S.hacc, 1, out, dtype);
}

#ifndef TILD_PART_F64
hipError_t launch_force_vjp_ik(const Launch& L, DeviceState& S, const void* lam, void* out, int dtype) {
    if (S.n == 0) return hipSuccess;
    if (L.order < 2 || L.force_ad) return hipErrorInvalidValue;
    hipError_t e = launch_bead_vectors(L, S, S.vdir, 0, const_cast<void*>(lam), dtype);
    // the gradient planes of the counts at the current positions (noise off)
    if (e == hipSuccess) e = launch_spread_xy(L, S);
    if (e == hipSuccess) e = launch_z_kmul(L, S, false);
    if (e != hipSuccess) return e;
    if (L.precision != 0) return second_vjp_f64(L, S, out, dtype);
    return L.plane_block == 256 ? vjp_b<float, 256>(L, S, out, dtype) : vjp_b<float, 512>(L, S, out, dtype);
}
#else
hipError_t second_vjp_f64(const Launch& L, DeviceState& S, void* out, int dtype) {
    return L.plane_block == 256 ? vjp_b<double, 256>(L, S, out, dtype) : vjp_b<double, 512>(L, S, out, dtype);
}
#endif

template <typename T> static hipError_t attr_second(const Launch& L, size_t lds) {
    hipError_t e = hipSuccess;
    auto set = [&](const void* f) {
        if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    };
    with_order(L.order, [&](auto Pc) {
        constexpr int P = decltype(Pc)::value;
        if (L.plane_block == 256) {
            if constexpr (P >= 3) {
                set((const void*)k_xy_c2r<T, 256, P, true, false, true>);
                set((const void*)k_spread_xy<T, 256, P, false, true>);
            }
            if constexpr (P >= 2) {
                set((const void*)k_xy_c2r<T, 256, P, true, false, false, true>);
                set((const void*)k_xy_c2r<T, 256, P, false, false, false, false, 1>);
                set((const void*)k_xy_c2r<T, 256, P, false, false, false, false, 2>);
                set((const void*)k_spread_xy<T, 256, P, false, true, false, true>);
            }
            set((const void*)k_spread_xy<T, 256, P, false, false, true>);
        } else {
            if constexpr (P >= 3) {
                set((const void*)k_xy_c2r<T, 512, P, true, false, true>);
                set((const void*)k_spread_xy<T, 512, P, false, true>);
            }
            if constexpr (P >= 2) {
                set((const void*)k_xy_c2r<T, 512, P, true, false, false, true>);
                set((const void*)k_xy_c2r<T, 512, P, false, false, false, false, 1>);
                set((const void*)k_xy_c2r<T, 512, P, false, false, false, false, 2>);
                set((const void*)k_spread_xy<T, 512, P, false, true, false, true>);
            }
            set((const void*)k_spread_xy<T, 512, P, false, false, true>);
        }
    });
    return e;
}

#ifndef TILD_PART_F64
hipError_t configure_second_attributes(const Launch& L, size_t lds) {
    return L.precision == 0 ? attr_second<float>(L, lds) : second_attr_f64(L, lds);
}
#else
hipError_t second_attr_f64(const Launch& L, size_t lds) { return attr_second<double>(L, lds); }
#endif

}  // namespace tild

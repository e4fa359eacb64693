// Host-side launch interface of the TILD kernels (implemented in tild_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "tild_fft.h"

namespace tild {

// Physical constants of one context, passed by value to kernels.
struct Phys {
    double lx, ly, lz;
    double a2;          // smear_a^2
    double chi, kappa;  // interaction parameters
    double inv_n;       // 1 / N
    double bond_k;
    double mob_dt;      // dt / gamma
    double noise_amp;   // sqrt(2 kT dt / gamma)
    uint64_t seed;
    int com_correct;
};

// Everything a step needs on the device.
struct DeviceState {
    uint4* pos;            // [n] {qx, qy, qz, species}: current positions
    uint4* pos_next;       // [n] positions after the step being computed (swapped with pos by the host)
    uint32_t* qshift;      // [4] global fixed-point shift (centre-of-mass correction); x = (q - qshift) L / 2^32
    uint32_t* qshift_next; // [4] shift after the step being computed
    int32_t* bond_off;     // [n + 1]
    int32_t* bond_nbr;     // [2 n_bonds]
    void* dens;            // real [2][mz][my][mx]
    void* spec;            // complex [2][mz][my][hx]
    void* zout;            // complex [4][mz][my][hx]: z-inverted phi_A, phi_B, then ik_z phi_A, ik_z phi_B
    void* grad;            // real [2][3][mz][my][mx]
    void* tw;              // complex twiddle tables
    double* epart;         // [n_zblocks][5] energy partials of the k-space pass
    double* bpart;         // [n_bblocks][4] bond energy / virial partials
    unsigned long long* com_acc;  // [4]: int64 displacement sums (x, y, z) and a block counter
    uint32_t* flag;        // [1] non-finite latch
    double* eout;          // [8] reduced energies
    long long n;
    long long n_a, n_b;
};

struct Launch {
    hipStream_t stream;
    int precision;   // 0 float, 1 double
    int order;       // P
    Dims d;
    FftPlan px, py, pz;
    int plane_block;  // threads per workgroup of the plane passes
    int z_cols;       // columns per workgroup of the z pass
    int z_block;
    int n_zblocks;
    int n_bblocks;
    Phys ph;
};

// Launch helpers; each returns the hipError_t of the launch.
hipError_t launch_fill_mean(const Launch& L, DeviceState& S);
hipError_t launch_spread(const Launch& L, DeviceState& S);
hipError_t launch_xy_r2c(const Launch& L, DeviceState& S);
hipError_t launch_z_kmul(const Launch& L, DeviceState& S, bool energy_only);
hipError_t launch_xy_c2r(const Launch& L, DeviceState& S);
// mode 0: Euler-Maruyama step; mode 1: write forces (parts) to out (out_dtype 0 float / 1 double)
hipError_t launch_gather(const Launch& L, DeviceState& S, int mode, uint64_t step, void* out, int out_dtype,
                         unsigned parts);
hipError_t launch_bond_energy(const Launch& L, DeviceState& S);
hipError_t launch_reduce_energy(const Launch& L, DeviceState& S);
hipError_t launch_set_positions(const Launch& L, DeviceState& S, const void* xyz, int dtype);
hipError_t launch_get_positions(const Launch& L, DeviceState& S, void* xyz, int dtype);
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t stream);

// Largest dynamic LDS a plane / z workgroup needs (bytes), used for validation.
size_t plane_lds_bytes(const Launch& L);
size_t z_lds_bytes(const Launch& L);
hipError_t configure_kernel_attributes(const Launch& L);

}  // namespace tild

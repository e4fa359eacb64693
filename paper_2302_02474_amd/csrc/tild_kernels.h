// Host-side launch interface of the TILD kernels (implemented in tild_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "tild_fft.h"

namespace tild {

constexpr int kZBlock = 512;         // threads per workgroup of the z pass
constexpr int kEpart = 9;            // energy partials per z-pass workgroup
constexpr int kScanBins = 1024;      // bins per workgroup of the bin scan
constexpr int kSmallPlaneBlock = 128;        // threads per plane workgroup of a batch's small planes
constexpr size_t kSmallPlaneLds = 20 * 1024;  // LDS bound of a small plane (eight workgroups per CU)
constexpr int kStepBeads = 2;        // beads per thread of the Euler-Maruyama update and the scatter

// Physical constants of one context, passed by value to kernels.
struct Phys {
    double lx, ly, lz;
    double qx, qy, qz;  // 2^32 / L per axis: fixed-point units per length
    double a2;          // smear_a^2
    double chi, kappa;  // interaction parameters
    double inv_n;       // 1 / N
    double bond_k;
    double mob_dt;      // coefficient of F in a step's displacement: dt / gamma (EM) or b dt^2 / m (GJF)
    double noise_amp;   // coefficient of the unit noise: sqrt(2 kT dt / gamma) (EM) or
                        // (b dt / 2m) sqrt(2 gamma kT dt) (GJF, times xi_n + xi_{n+1})
    int gjf;            // GJF integrator: D_{n+1} = a D_n + mob_dt F + noise_amp (xi_n + xi_{n+1})
    double gjf_a;       // a = (1 - c)/(1 + c), c = gamma dt / 2m
    double gjf_vs;      // sqrt(b) dt: D = gjf_vs u for the half-step velocity u
    int elec;           // per-species charges with a Coulomb kernel
    double qa, qb;      // charges of A and B beads
    double lb4v;        // 4 pi l_B / V
    double ae2;         // a_e^2, charge smearing
    double mean_a, mean_b;  // N_A / M, N_B / M: subtracted from the counts
    double wmax;            // largest single-bead weight of one grid point, (max B_P)^3
    double u0;              // kernel at k = 0 (1 for the analytic kernel)
    int sampled;            // the kernel is the node-sampled one
    uint64_t seed;
    int com_correct;
};

// Device memory of one context.
//
// Beads live in "sorted order": grouped by bin key
//   key = (species * mz + g0z) * my + g0y,
// g0 the first grid index of the bead's assignment stencil, so that the
// beads touching one z-plane of one species occupy a few contiguous slot
// ranges.  A bead is a uint4 {qx, qy, qz, (abi_id << 1) | species}; qx.. are
// 32-bit fixed-point box fractions; the true coordinate is
// (q - qshift) * L / 2^32.  Every step the update kernel writes the new
// positions in the old order together with each bead's new key and its rank
// within the key's bin, a scan turns bin counts into bin starts, and a
// scatter moves beads into the new order, re-maps bond partner slots and
// stores each bead's bond force.
struct DeviceState {
    uint4* pos;           // [n] sorted beads
    uint4* pos_tmp;       // [n] beads in the previous order (new positions or ABI input)
    uint4* grec;          // [n] grid records of the sorted beads {x, y, z, id << 1 | species} (grid_record;
                          // single precision only): first stencil node and 24-bit fraction per axis
    uint2* kr;            // [n] {bin key, rank within the bin} of pos_tmp[j]
    void* fbond;          // [n][4] harmonic bond force of sorted bead j {Fx, Fy, Fz, 0} (working precision)
    void* vel;            // GJF only: [n][4] half-step velocity of sorted bead j {ux, uy, uz, 0}
    void* vel_tmp;        // GJF only: the same in the order of pos_tmp
    void* vdir;           // [n][4] direction v of a Hessian-vector product, sorted order
    void* hacc;           // [n][4] accumulated H v (or J^T v), sorted order
    void* field;          // [2][mz][my][mx] working-precision grid field (order >= 2): the adjoint's psi
    double* adj;          // [n][3] float64 work array of the adjoint step (order >= 2)
    double* apart;        // [n_bblocks][4] float64 block partial sums of the adjoint step
    uint32_t* counts;     // [nbins] bin occupancy (kept zero between uses)
    uint32_t* bin_start;  // [nbins + 1] first sorted slot of each bin
    unsigned long long* scan_status;  // [ntiles + 1] look-back status words of the bin scan, then its ticket
    int32_t* nbr;         // [n][deg] bond partners of sorted slot j as sorted slots, -1 padded
    int32_t* nbr_old;     // [n][deg] partners in the previous order
    int32_t* nbr_abi;     // [n][deg] partners in ABI order (static)
    uint32_t* types_abi;  // [n] species in ABI order (static)
    uint32_t* qshift;       // [4] fixed-point centre-of-mass shift
    uint32_t* qshift_next;  // [4] shift after the step being computed
    void* spec;           // complex [2][mz][my][hx] half spectra of the counts
    void* zout;           // complex [4][mz][my][hx]: z-inverted Phi_A, Phi_B, then ik_z Phi_A, ik_z Phi_B
    void* fpart;          // real [3][P][n] non-bonded force partials: axis, stencil plane offset, sorted bead
    void* tw;             // complex twiddle tables
    double* utab;         // [mx + my + mz] per-axis factors of the kernel u^ (index n along each axis)
    double* vtab;         // [mx + my + mz] per-axis factors of exp(-a^2 k^2) (virial); utab's array when equal
    double* epart;        // [n_zblocks][5] energy partials of the k-space pass
    long long* bpart;     // [n_bblocks][4] bond energy / virial partials (32.32 fixed point)
    long long* noise_part;  // [max(n_bblocks, 2 mz)][3] per-256-bead-block sums of a step's Gaussian increments
                            // (32.32 fixed point)
    long long* fsum_part;   // [2 mz][3] per-plane sums of the non-bonded forces (exact-gradient route)
    uint32_t* flag;       // [1] bit 0: non-finite value; bit 2: a grid plane too dense for the fixed-point spread
    double* eout;         // [16] reduced energies, virial, parameter gradients
    long long n;
    long long n_a, n_b;
    int deg;              // bond slots per bead (maximum degree)
    int noise_step;       // set while stepping: the k-space pass forms qshift_next from the noise sums
    int nbins;            // 2 * mz * my
};

// One member of a batch of independent contexts stepped together: what the
// batched kernels read from its context.  The pointer pairs (qshift,
// qshift_next) and (nbr, nbr_old) are those at the start of a batch call;
// at step s of the call the kernels take them swapped when s is odd.
struct RepDesc {
    Dims d;
    FftPlan px, py, pz;
    Phys ph;
    DeviceState S;   // S.scan_status points at the batch's own status words for this member
    int z_cols;
    int n_zblocks;
    int ntiles;      // bin scan tiles
    uint64_t step0;  // the member's step counter at the start of the call
};

// Work-unit maps of a batched launch: entry g = (member << 16) | local unit.
struct BatchMaps {
    const RepDesc* reps;
    const uint32_t* plane;  // spread units: (z, species) planes, 2 mz per member
    const uint32_t* c2r;    // inverse plane units: (z, species, axis), 6 mz per member
    const uint32_t* zcol;   // z-pass column blocks, n_zblocks per member
    const uint32_t* bead;   // 256-bead blocks, ceil(n / 256) per member
    const uint32_t* tile;   // bin scan tiles, ntiles per member
    int n_plane, n_c2r, n_zcol, n_bead, n_tile;
    unsigned long long* ticket;  // the batch's scan ticket
    int plane_block;  // threads per plane workgroup (256 or 512) for the members of large planes
    // the last n_plane_small / n_c2r_small units of plane / c2r belong to members of small planes, launched
    // separately with kSmallPlaneBlock threads and lds_small bytes of LDS, so more of their workgroups fit a CU
    int n_plane_small, n_c2r_small;
    size_t lds_small;
    int deg;  // the members' common partner-table width when it is 1..4 (partners held in registers), else 0
};

struct Launch {
    hipStream_t stream;
    int precision;   // 0 float, 1 double
    int order;       // P
    Dims d;
    FftPlan px, py, pz;
    int plane_block;  // threads per workgroup of the inverse plane pass
    int force_ad;     // exact-gradient route: potential planes, weight derivatives (else the ik route)
    int spread_block; // threads per workgroup of the fused spread + forward plane pass
    int z_cols;       // columns per workgroup of the z pass
    int z_block;
    int n_zblocks;
    int n_bblocks;
    int cu_count;     // compute units of the device
    Phys ph;
};

// What the spread and interpolation kernels read per sorted bead: grid
// records in single precision, fixed-point positions in double precision.
inline const uint4* bead_src(const Launch& L, const DeviceState& S) { return L.precision == 0 ? S.grec : S.pos; }

// Launch helpers; each returns the hipError_t of the launch.
hipError_t launch_spread_xy(const Launch& L, DeviceState& S);
// energy_only: energy partials only; with_energy: energy partials and the
// inverse spectra
hipError_t launch_z_kmul(const Launch& L, DeviceState& S, bool energy_only, bool with_energy = false);
// route: -1 the context's, 0 ik, 1 exact gradient
hipError_t launch_xy_c2r(const Launch& L, DeviceState& S, int route = -1);
// mode 0: one step of the context's integrator (Euler-Maruyama, or GJF when
// ph.gjf, which also writes vel_tmp) with the shift the k-space pass formed in
// qshift_next (writes pos_tmp, kr, counts);
// mode 1: write out_sign * forces (parts) to out[abi id] (out_dtype 0 float / 1 double)
hipError_t launch_update(const Launch& L, DeviceState& S, int mode, uint64_t step, void* out, int out_dtype,
                         unsigned parts, double out_sign = 1.0);
hipError_t launch_bin_scan(const Launch& L, DeviceState& S);
// noise_step >= 0: also the per-block noise sums of step noise_step (into noise_part)
hipError_t launch_scatter(const Launch& L, DeviceState& S, const int32_t* nbr_src, int64_t noise_step = -1);
// per-block noise sums of step `step` (into noise_part), from the beads' ids in pos
hipError_t launch_noise_sum(const Launch& L, DeviceState& S, uint64_t step);
hipError_t launch_bond_energy(const Launch& L, DeviceState& S);
hipError_t launch_reduce_energy(const Launch& L, DeviceState& S);
// ABI-order input -> pos_tmp, key, rank (qshift reset to 0)
hipError_t launch_place(const Launch& L, DeviceState& S, const void* xyz, int dtype);
hipError_t launch_get_positions(const Launch& L, DeviceState& S, void* xyz, int dtype);
// GJF velocities, ABI order [n][3] of dtype: op 0 set (v -> vel), op 1 get
// (vel -> v), op 2 vel (sorted) -> vel_tmp in ABI order (v unused), before a
// re-placement of the beads
hipError_t launch_velocities(const Launch& L, DeviceState& S, int op, void* v, int dtype);

// Hessian-vector product of the total energy at the current positions:
// v ([n][3] ABI order, dtype) -> out ([n][3] ABI order, dtype), through vdir
// and hacc (order >= 3).
hipError_t launch_hvp(const Launch& L, DeviceState& S, const void* v, void* out, int dtype);
// Transposed Jacobian of the ik-route force (non-bonded and bonds) at the
// current positions applied to lam ([n][3] ABI order, dtype) -> out ([n][3]
// ABI order, dtype), through vdir, hacc and field (order >= 2, ik route).
hipError_t launch_force_vjp_ik(const Launch& L, DeviceState& S, const void* lam, void* out, int dtype);
// [n][3] ABI-order vector operations of the adjoint step (v of dtype 0 float / 1 double, w float64
// unless stated): kMean out[0..2] = mean of v; kProject w (dtype) = v - out[0..2] (out NULL: copy);
// kDotAdd out[0] += alpha v . w; kAxpy v += alpha w; kScale v *= alpha.  Sums in a fixed order (apart).
enum class AdjointOp { kMean, kProject, kDotAdd, kAxpy, kScale };
hipError_t launch_adjoint_vectors(const Launch& L, DeviceState& S, AdjointOp op, void* v, void* w, int dtype,
                                  double alpha, double* out);
// Counts c_K(g) ([2][mz][my][mx], x fastest, working precision) to device memory.
hipError_t launch_counts(const Launch& L, DeviceState& S, void* out);
// Forces -sum_g grad W_i(g) psi_{s_i}(g) of a given field psi ([2][mz][my][mx],
// working precision, device) to out ([n][3] ABI order, dtype); order >= 2.
hipError_t launch_field_forces(const Launch& L, DeviceState& S, const void* field, void* out, int dtype);
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t stream);

// One step of every member of a batch (ik route, Euler-Maruyama, all members
// of the same precision, order and flags as L), one launch per kernel; s is
// the step's index within the call (its parity selects the pointer pairs).
// lds_plane / lds_z: the largest dynamic LDS any member needs.
hipError_t launch_batch_step(const Launch& L, const BatchMaps& B, int s, size_t lds_plane, size_t lds_z);
// every member's per-block noise sums of its current step (before the first batched step of a call)
hipError_t launch_batch_noise(const Launch& L, const BatchMaps& B);
hipError_t configure_batch_attributes(const Launch& L, size_t lds_plane, size_t lds_z);

// Dynamic LDS a plane / z workgroup needs (bytes), used for validation.
size_t plane_lds_bytes(const Launch& L);
size_t z_lds_bytes(const Launch& L);
hipError_t configure_kernel_attributes(const Launch& L);
hipError_t configure_plane_attributes(const Launch& L, size_t lds);
hipError_t configure_second_attributes(const Launch& L, size_t lds);
// [n][4] sorted-order vectors <-> [n][3] ABI-order arrays of dtype: op 0 ABI -> sorted, op 1 sorted -> ABI
hipError_t launch_bead_vectors(const Launch& L, DeviceState& S, void* sorted, int op, void* v, int dtype);

}  // namespace tild

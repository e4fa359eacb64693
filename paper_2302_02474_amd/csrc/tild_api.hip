// C ABI of libtild: context creation, parameter validation, device memory,
// step orchestration, I/O conversions and error reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "tild.h"
#include "tild_kernels.h"

#define TILD_API extern "C" __attribute__((visibility("default")))

using namespace tild;

namespace {

thread_local std::string g_create_error;

enum Slot { kSpreadXy = 0, kZKmul, kXyC2r, kUpdate, kBinScan, kScatter, kNumSlots };
static_assert(kNumSlots == TILD_NUM_KERNELS, "slot table");
const char* kSlotNames[kNumSlots] = {"spread_fft_xy", "fft_z_kmul", "fft_xy_c2r_gather",
                                     "update_em_keys", "bin_scan",  "bin_scatter_bonds"};

// Uncentred cardinal B-spline M_k(s) (support [0, k)), by its recursion.
double uncentred_bspline(int k, double s) {
    if (k == 1) return (s >= 0.0 && s < 1.0) ? 1.0 : 0.0;
    return (s * uncentred_bspline(k - 1, s) + (k - s) * uncentred_bspline(k - 1, s - 1.0)) / (k - 1);
}
constexpr int kMaxDegree = 64;

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

bool smooth235(int n) {
    if (n < 1) return false;
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

// Radix passes for one length: as many 8s as possible, then 4, 2, 3, 5.
// Lengths 64, 128 and 256 also get the two-pass shape (8 x 8, 16 x 8,
// 16 x 16), whose table starts at tw2_offset.
bool make_plan(int n, int tw_offset, int tw2_offset, FftPlan& pl) {
    std::memset(&pl, 0, sizeof(pl));
    pl.n = n;
    pl.tw = tw_offset;
    pl.tw2 = tw2_offset;
    pl.r1 = n == 64 ? 8 : ((n == 128 || n == 256) ? 16 : 0);
    int r = n, k = 0;
    auto push = [&](int R) {
        if (k >= kMaxRadixStages) return false;
        pl.codes |= (uint32_t)R << (4 * k++);
        r /= R;
        return true;
    };
    while (r % 8 == 0)
        if (!push(8)) return false;
    while (r % 4 == 0)
        if (!push(4)) return false;
    while (r % 2 == 0)
        if (!push(2)) return false;
    while (r % 3 == 0)
        if (!push(3)) return false;
    while (r % 5 == 0)
        if (!push(5)) return false;
    pl.nst = k;
    return r == 1;
}

}  // namespace

struct tild_ctx {
    tild_params p{};
    int device = 0;
    Launch L{};
    DeviceState S{};
    int64_t step = 0;
    int64_t noise_ready = -1;  // the step whose per-block noise sums noise_part holds (-1: none)
    bool have_pos = false;
    std::string err;
    void* staging = nullptr;  // device [n][3] doubles for host transfers
    std::vector<void*> allocs;
    int64_t n_bonds = 0;

    int fail(int code, const std::string& msg) {
        err = msg;
        return code;
    }
    int hip_fail(hipError_t e, const char* what) {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return TILD_EHIP;
    }
    // Device memory: hipMalloc, carved from a caller workspace, or (measure)
    // only counted.  Every buffer starts on a 256-byte boundary.
    char* ws_base = nullptr;
    size_t ws_size = 0, ws_used = 0;
    bool measure = false;
    hipError_t alloc(void** p, size_t bytes) {
        if (bytes == 0) bytes = 16;
        if (measure || ws_base) {
            const size_t off = (ws_used + 255) / 256 * 256;
            if (!measure && off + bytes > ws_size) return hipErrorOutOfMemory;
            *p = measure ? nullptr : ws_base + off;
            ws_used = off + bytes;
            return hipSuccess;
        }
        hipError_t e = hipMalloc(p, bytes);
        if (e == hipSuccess) allocs.push_back(*p);
        return e;
    }
};

namespace {

int validate(const tild_params* p, int64_t n, std::string& why) {
    if (!p) return why = "params is NULL", TILD_EINVAL;
    if (n < 0 || n >= (int64_t)1 << 31) return why = "n_beads must be in [0, 2^31)", TILD_EINVAL;
    for (int a = 0; a < 3; ++a) {
        if (!(p->box[a] > 0.0) || !std::isfinite(p->box[a])) return why = "box edges must be finite and > 0", TILD_EINVAL;
        if (p->grid[a] < 2 || p->grid[a] > 256 || !smooth235(p->grid[a]))
            return why = "grid sizes must be in [2, 256] and products of 2, 3 and 5", TILD_EINVAL;
        if (p->order > p->grid[a]) return why = "order must not exceed any grid size", TILD_EINVAL;
    }
    if (p->order < 1 || p->order > 7) return why = "order must be in [1, 7]", TILD_EINVAL;
    if (!(p->smear_a >= 0.0) || !std::isfinite(p->smear_a)) return why = "smear_a must be finite and >= 0", TILD_EINVAL;
    if (!std::isfinite(p->chi) || !std::isfinite(p->kappa) || !std::isfinite(p->bond_k))
        return why = "chi, kappa and bond_k must be finite", TILD_EINVAL;
    if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return why = "dt must be finite and > 0", TILD_EINVAL;
    if (!(p->gamma > 0.0) || !std::isfinite(p->gamma)) return why = "gamma must be finite and > 0", TILD_EINVAL;
    if (!(p->kT >= 0.0) || !std::isfinite(p->kT)) return why = "kT must be finite and >= 0", TILD_EINVAL;
    if (p->precision != TILD_FP32 && p->precision != TILD_FP64) return why = "precision must be TILD_FP32 or TILD_FP64", TILD_EINVAL;
    if (p->flags & ~(TILD_COM_CORRECT | TILD_POTENTIAL_SAMPLED | TILD_DETERMINISTIC | TILD_FORCE_AD |
                     TILD_INTEGRATOR_GJF))
        return why = "unknown flag bits", TILD_EINVAL;
    if ((p->flags & TILD_FORCE_AD) && p->order < 2) return why = "TILD_FORCE_AD needs order >= 2", TILD_EINVAL;
    if ((p->flags & TILD_INTEGRATOR_GJF) && !(p->mass >= 0.0 && std::isfinite(p->mass)))
        return why = "mass must be finite and > 0 (0 reads as 1)", TILD_EINVAL;
    if (!std::isfinite(p->charge[0]) || !std::isfinite(p->charge[1]) || !(p->bjerrum >= 0.0) ||
        !std::isfinite(p->bjerrum) || !(p->charge_smear >= 0.0) || !std::isfinite(p->charge_smear))
        return why = "charge must be finite, bjerrum and charge_smear finite and >= 0", TILD_EINVAL;
    if ((p->flags & TILD_POTENTIAL_SAMPLED) && !(p->smear_a > 0.0))
        return why = "TILD_POTENTIAL_SAMPLED needs smear_a > 0", TILD_EINVAL;
    return TILD_OK;
}

// Smallest power-of-two lane group (<= 64, >= min_g) for which every radix
// pass of `pl` fits the per-lane register budget of the line transform; the
// two-pass shapes have fixed groups (n/16 lanes for 128 and 256, 8 for 64).
int choose_group(const FftPlan& pl, int min_g) {
    if (pl.r1) {
        const int G = pl.n == 64 ? 8 : pl.n / 16;
        return G >= min_g ? G : 0;
    }
    for (int G = 1; G <= 64; G <<= 1) {
        if (G < min_g) continue;
        bool ok = true;
        for (int st = 0; st < pl.nst; ++st) {
            const int R = pl.radix(st), bpl = pl.n / R;
            if ((bpl + G - 1) / G > kFftRegElems / R) ok = false;
        }
        if (ok) return G;
    }
    return 0;
}

// Choose workgroup shapes; false if the grid does not fit the kernels' limits.
bool choose_shapes(Launch& L, std::string& why) {
    const Dims& d = L.d;
    const size_t lds_max = 160 * 1024;
    const int pair_items = kPairItems;  // row-pair (un)packing items per lane in the plane kernels
    L.px.group = choose_group(L.px, (d.mx + pair_items - 1) / pair_items);
    L.py.group = choose_group(L.py, 1);
    L.pz.group = choose_group(L.pz, 1);
    if (!L.px.group || !L.py.group || !L.pz.group) {
        why = "internal: no lane group fits a transform length";
        return false;
    }
    const long long need = std::max((long long)d.npair * L.px.group, (long long)d.hx * L.py.group);
    // measured on MI355X at 128^2 planes: the fused spread prefers 1024 threads, the inverse pass 512
    L.plane_block = need <= 256 ? 256 : 512;
    L.spread_block = need <= 256 ? 256 : (L.precision == 1 ? 512 : 1024);
    if (plane_lds_bytes(L) > lds_max) {
        why = "grid plane does not fit one workgroup's LDS in this precision";
        return false;
    }
    // z pass: columns per workgroup chosen to minimise (rounds of resident workgroups) x (columns each),
    // with at most two 512-thread workgroups per CU (registers) and the LDS they need
    L.z_block = kZBlock;
    {
        int best_cb = 0;
        long long best = 0;
        for (int cb = 1; cb <= 32; ++cb) {
            L.z_cols = cb;
            const size_t lds = z_lds_bytes(L);
            if (lds > lds_max) break;
            const long long per_cu = std::min<long long>(2, (long long)(lds_max / lds));
            const long long slots = per_cu * L.cu_count;
            const long long nblk = (d.hplane + cb - 1) / cb;
            const long long cost = ((nblk + slots - 1) / slots) * cb;
            if (best_cb == 0 || cost < best || (cost == best && cb > best_cb)) {
                best = cost;
                best_cb = cb;
            }
        }
        if (best_cb == 0) {
            why = "z columns do not fit LDS";
            return false;
        }
        L.z_cols = best_cb;
    }
    L.n_zblocks = (int)((d.hplane + L.z_cols - 1) / L.z_cols);
    return true;
}

int check_flag(tild_ctx* c) {
    uint32_t f = 0;
    hipError_t e = hipMemcpyAsync(&f, c->S.flag, sizeof(f), hipMemcpyDeviceToHost, c->L.stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->L.stream);
    if (e != hipSuccess) return c->hip_fail(e, "synchronize");
    if (f) {
        e = hipMemsetAsync(c->S.flag, 0, sizeof(uint32_t), c->L.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->L.stream);
        if (e != hipSuccess) return c->hip_fail(e, "clear flag");
        std::string why;
        if (f & 1u) why += "non-finite force, displacement or position detected; ";
        if (f & 4u) why += "a grid plane is too dense for the fixed-point spread; ";
        if (f & 8u) why += "internal: a bead was found outside its bin; ";
        if (f & 16u) why += "internal: the bin prefix scan gave up waiting for a preceding tile; ";
        return c->fail((f & 24u) ? TILD_EHIP : TILD_ENONFINITE, why);
    }
    return TILD_OK;
}

// Forces on the mesh up to the gradient fields (no bead update).
hipError_t mesh_forward(tild_ctx* c, bool energy_only) {
    hipError_t e = launch_spread_xy(c->L, c->S);
    if (e == hipSuccess) e = launch_z_kmul(c->L, c->S, energy_only);
    if (e == hipSuccess && !energy_only) e = launch_xy_c2r(c->L, c->S);
    return e;
}

// Sort the beads held in pos_tmp (keys and ranks already counted) into pos,
// translating bond partners given as slots of pos_tmp's order.
hipError_t sort_beads(tild_ctx* c, const int32_t* nbr_src) {
    hipError_t e = launch_bin_scan(c->L, c->S);
    if (e == hipSuccess) e = launch_scatter(c->L, c->S, nbr_src);
    if (e == hipSuccess) std::swap(c->S.nbr, c->S.nbr_old);
    return e;
}

int run_steps(tild_ctx* c, int64_t n_steps, std::vector<hipEvent_t>* ev) {
    for (int64_t s = 0; s < n_steps; ++s) {
        hipError_t e = hipSuccess;
        auto mark = [&](int slot, int which) {
            if (ev && e == hipSuccess) e = hipEventRecord((*ev)[(size_t)(s * kNumSlots + slot) * 2 + which], c->L.stream);
        };
        // the step's noise sums, for its centre-of-mass shift: left by the previous step's scatter, else
        // drawn here
        if (c->noise_ready != c->step && e == hipSuccess) e = launch_noise_sum(c->L, c->S, (uint64_t)c->step);
        c->noise_ready = -1;
        mark(kSpreadXy, 0);
        c->S.noise_step = 1;
        if (e == hipSuccess) e = launch_spread_xy(c->L, c->S);
        mark(kSpreadXy, 1);
        mark(kZKmul, 0);
        if (e == hipSuccess) e = launch_z_kmul(c->L, c->S, false);  // also forms the new shift
        c->S.noise_step = 0;
        mark(kZKmul, 1);
        mark(kXyC2r, 0);
        if (e == hipSuccess) e = launch_xy_c2r(c->L, c->S);
        mark(kXyC2r, 1);
        mark(kUpdate, 0);
        if (e == hipSuccess) e = launch_update(c->L, c->S, 0, (uint64_t)c->step, nullptr, 0, 0);
        mark(kUpdate, 1);
        if (e == hipSuccess) std::swap(c->S.qshift, c->S.qshift_next);
        mark(kBinScan, 0);
        if (e == hipSuccess) e = launch_bin_scan(c->L, c->S);
        mark(kBinScan, 1);
        mark(kScatter, 0);
        if (e == hipSuccess) e = launch_scatter(c->L, c->S, c->S.nbr, c->step + 1);  // also the next step's noise sums
        mark(kScatter, 1);
        if (e == hipSuccess) std::swap(c->S.nbr, c->S.nbr_old);
        if (e != hipSuccess) return c->hip_fail(e, "step launch");
        ++c->step;
        c->noise_ready = c->step;
    }
    return TILD_OK;
}

}  // namespace

namespace {

// Per-axis kernel factors, index n along each axis: u^(n) = t_x(n_x) t_y(n_y)
// t_z(n_z).  vt: t(n) = exp(-a^2 k_n^2), k_n = 2 pi n' / L with n' the signed
// index.  ut: the kernel's factors, vt itself, or with TILD_POTENTIAL_SAMPLED
// t(n) = h sum_g g(d_g) cos(2 pi n g / M), g the 1-D factor of the Gaussian u_G
// (variance 2 a^2) at the minimum-image separation d_g of node g.
void kernel_tables(const tild_params& p, const Dims& d, std::vector<double>& ut, std::vector<double>& vt) {
    const bool sampled = (p.flags & TILD_POTENTIAL_SAMPLED) != 0;
    ut.clear();
    vt.clear();
    for (int a = 0; a < 3; ++a) {
        const int m = a == 0 ? d.mx : (a == 1 ? d.my : d.mz);
        const double len = p.box[a], h = len / m, s2 = 2.0 * p.smear_a * p.smear_a;
        for (int nn = 0; nn < m; ++nn) {
            const double k = 2.0 * M_PI * (double)(nn > m / 2 ? nn - m : nn) / len;
            vt.push_back(std::exp(-p.smear_a * p.smear_a * k * k));
            if (sampled) {
                double acc = 0.0;
                for (int g = 0; g < m; ++g) {
                    const double dg = (double)(g > m / 2 ? g - m : g) * h;
                    acc += std::exp(-dg * dg / (2.0 * s2)) * std::cos(2.0 * M_PI * (double)nn * g / m);
                }
                ut.push_back(h * acc / std::sqrt(2.0 * M_PI * s2));
            }
        }
    }
    if (!sampled) ut = vt;
}

// tild_create, or with `measure` the device bytes it would need (types may
// then be NULL; nothing touches the device).
int create_impl(const tild_params* params, int64_t n_beads, const int32_t* types, int64_t n_bonds,
                const int32_t* bonds, void* workspace, size_t workspace_bytes, void* hip_stream, tild_ctx** out,
                size_t* measure) {
    if (!out && !measure) {
        g_create_error = "out is NULL";
        return TILD_EINVAL;
    }
    if (out) *out = nullptr;
    if (workspace && (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)) {
        g_create_error = "workspace must be 256-byte aligned";
        return TILD_EINVAL;
    }
    std::string why;
    int rc = validate(params, n_beads, why);
    if (rc != TILD_OK) {
        g_create_error = why;
        return rc;
    }
    if (n_beads > 0 && !types && !measure) {
        g_create_error = "types is NULL";
        return TILD_EINVAL;
    }
    if (n_bonds < 0 || (n_bonds > 0 && !bonds) || n_bonds >= (int64_t)1 << 30) {
        g_create_error = "invalid bond list";
        return TILD_EINVAL;
    }
    // Host-side checks and bond CSR (both ends of every bond).
    int64_t n_a = 0, n_b = 0;
    for (int64_t i = 0; types && i < n_beads; ++i) {
        if (types[i] == 0) ++n_a;
        else if (types[i] == 1) ++n_b;
        else {
            g_create_error = "types must be 0 (A) or 1 (B)";
            return TILD_EINVAL;
        }
    }
    std::vector<int32_t> off((size_t)n_beads + 1, 0), nbr((size_t)(2 * n_bonds));
    for (int64_t b = 0; b < n_bonds; ++b) {
        const int32_t i = bonds[2 * b], j = bonds[2 * b + 1];
        if (i < 0 || j < 0 || i >= n_beads || j >= n_beads || i == j) {
            g_create_error = "bond index out of range or self-bond at bond " + std::to_string(b);
            return TILD_EINVAL;
        }
        ++off[(size_t)i + 1];
        ++off[(size_t)j + 1];
    }
    for (int64_t i = 0; i < n_beads; ++i) off[(size_t)i + 1] += off[(size_t)i];
    {
        std::vector<int32_t> fill(off.begin(), off.end() - 1);
        for (int64_t b = 0; b < n_bonds; ++b) {
            const int32_t i = bonds[2 * b], j = bonds[2 * b + 1];
            nbr[(size_t)fill[(size_t)i]++] = j;
            nbr[(size_t)fill[(size_t)j]++] = i;
        }
    }

    int deg = 0;
    for (int64_t i = 0; i < n_beads; ++i) deg = std::max(deg, off[(size_t)i + 1] - off[(size_t)i]);
    if (deg > kMaxDegree) {
        g_create_error = "a bead has more than 64 bonds";
        return TILD_EINVAL;
    }
    // Partners of every bead at fixed width `deg`, -1 padded (ABI order).
    std::vector<int32_t> nbr_tab((size_t)n_beads * (size_t)deg, -1);
    for (int64_t i = 0; i < n_beads; ++i)
        for (int32_t k = off[(size_t)i]; k < off[(size_t)i + 1]; ++k)
            nbr_tab[(size_t)i * deg + (size_t)(k - off[(size_t)i])] = nbr[(size_t)k];

    tild_ctx* c = new (std::nothrow) tild_ctx();
    if (!c) {
        g_create_error = "out of host memory";
        return TILD_ENOMEM;
    }
    c->p = *params;
    c->n_bonds = n_bonds;
    c->measure = measure != nullptr;
    c->ws_base = static_cast<char*>(workspace);
    c->ws_size = workspace_bytes;
    Launch& L = c->L;
    L.stream = (hipStream_t)hip_stream;
    L.precision = params->precision;
    L.order = params->order;
    L.force_ad = (params->flags & TILD_FORCE_AD) ? 1 : 0;
    Dims& d = L.d;
    d.mx = params->grid[0];
    d.my = params->grid[1];
    d.mz = params->grid[2];
    d.hx = d.mx / 2 + 1;
    d.npair = (d.my + 1) / 2;
    d.npg = (d.my + params->order) / 2;
    d.ylines = (d.mx % 2 == 0 && d.hx > 1) ? d.hx - 1 : d.hx;
    d.swc = d.ylines % 16 == 0 ? d.ylines : 0;
    d.m = (long long)d.mx * d.my * d.mz;
    d.hplane = (long long)d.my * d.hx;
    d.lx = params->box[0];
    d.ly = params->box[1];
    d.lz = params->box[2];
    // the two-pass tables follow the plain ones, for the lengths that use them
    // ([n / r1][r1 + 1]: rows padded by one entry)
    int nt = d.mx + d.my + d.mz;
    bool planned = make_plan(d.mx, 0, nt, L.px);
    nt += L.px.r1 ? d.mx + d.mx / L.px.r1 : 0;
    planned = planned && make_plan(d.my, d.mx, nt, L.py);
    nt += L.py.r1 ? d.my + d.my / L.py.r1 : 0;
    planned = planned && make_plan(d.mz, d.mx + d.my, nt, L.pz);
    nt += L.pz.r1 ? d.mz + d.mz / L.pz.r1 : 0;
    d.ntw2 = nt - (d.mx + d.my + d.mz);
    // LDS plane: pair rows of 2 hxp complex, with room for P - 1 ghost columns
    // and P - 1 ghost rows past the periodic edge.  With the two-pass x
    // transform, hxp = 4 (mod 16): eight consecutive rows then start in four
    // bank groups two by two, which with the permuted intermediate order
    // leaves every LDS access of both passes (rows and columns) at the
    // two-cycle minimum of 64-bit accesses; otherwise hxp is odd, so that
    // consecutive pair rows start in different bank groups.
    {
        const int h0 = std::max(d.hx, (d.mx + params->order) / 2);
        d.hxp = L.px.r1 ? h0 + ((4 - h0 % 16) + 16) % 16 : (h0 | 1);
    }
    if (!planned) {
        g_create_error = "internal: radix plan";
        delete c;
        return TILD_EINVAL;
    }
    L.cu_count = 256;
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            L.cu_count = cus;
    }
    if (!choose_shapes(L, why)) {
        g_create_error = why;
        delete c;
        return TILD_EINVAL;
    }
    if (!measure && hipGetDevice(&c->device) != hipSuccess) {
        g_create_error = "no HIP device";
        delete c;
        return TILD_EHIP;
    }
    L.n_bblocks = (int)((n_beads + 255) / 256);
    if (L.n_bblocks < 1) L.n_bblocks = 1;
    Phys& ph = L.ph;
    ph.lx = d.lx;
    ph.ly = d.ly;
    ph.lz = d.lz;
    ph.qx = 4294967296.0 / d.lx;
    ph.qy = 4294967296.0 / d.ly;
    ph.qz = 4294967296.0 / d.lz;
    ph.a2 = params->smear_a * params->smear_a;
    ph.chi = params->chi;
    ph.kappa = params->kappa;
    ph.inv_n = n_beads > 0 ? 1.0 / (double)n_beads : 0.0;
    ph.bond_k = params->bond_k;
    ph.mob_dt = params->dt / params->gamma;
    ph.noise_amp = std::sqrt(2.0 * params->kT * params->dt / params->gamma);
    ph.seed = params->seed;
    ph.com_correct = (params->flags & TILD_COM_CORRECT) ? 1 : 0;
    ph.elec = (params->bjerrum != 0.0 && (params->charge[0] != 0.0 || params->charge[1] != 0.0)) ? 1 : 0;
    ph.qa = params->charge[0];
    ph.qb = params->charge[1];
    ph.lb4v = 4.0 * M_PI * params->bjerrum / (d.lx * d.ly * d.lz);
    ph.ae2 = params->charge_smear * params->charge_smear;
    ph.gjf = (params->flags & TILD_INTEGRATOR_GJF) ? 1 : 0;
    if (ph.gjf) {
        // GJF: c = gamma dt / 2m, a = (1 - c)/(1 + c), b = 1/(1 + c)
        const double m = params->mass > 0.0 ? params->mass : 1.0, dt = params->dt;
        const double cf = params->gamma * dt / (2.0 * m), b = 1.0 / (1.0 + cf);
        ph.gjf_a = (1.0 - cf) / (1.0 + cf);
        ph.gjf_vs = std::sqrt(b) * dt;
        ph.mob_dt = b * dt * dt / m;
        ph.noise_amp = b * dt / (2.0 * m) * std::sqrt(2.0 * params->gamma * params->kT * dt);
    }

    DeviceState& S = c->S;
    S.n = n_beads;
    S.n_a = n_a;
    S.n_b = n_b;
    S.deg = deg;
    S.nbins = 2 * d.mz * d.my;
    ph.mean_a = (double)n_a / (double)d.m;
    ph.mean_b = (double)n_b / (double)d.m;
    {
        const double peak = uncentred_bspline(params->order, 0.5 * params->order);
        ph.wmax = peak * peak * peak;
    }
    const size_t real_sz = L.precision == 0 ? 4 : 8;
    const size_t cplx_sz = 2 * real_sz;
    const size_t npos = (size_t)(n_beads > 0 ? n_beads : 1);
    hipError_t e = hipSuccess;
    auto A = [&](void** ptr, size_t bytes) {
        if (e == hipSuccess) e = c->alloc(ptr, bytes);
    };
    const size_t ntab = nbr_tab.size() > 0 ? nbr_tab.size() : 1;
    A((void**)&S.pos, npos * sizeof(uint4));
    A((void**)&S.pos_tmp, npos * sizeof(uint4));
    A((void**)&S.kr, npos * sizeof(uint2));
    if (L.precision == 0) A((void**)&S.grec, npos * sizeof(uint4));
    A(&S.fbond, npos * 4 * real_sz);
    if (ph.gjf) {
        A(&S.vel, npos * 4 * real_sz);
        A(&S.vel_tmp, npos * 4 * real_sz);
    }
    if (params->order >= 2) {  // Hessian-vector products (order >= 3), Jacobian products and adjoint steps
        A(&S.vdir, npos * 4 * real_sz);
        A(&S.hacc, npos * 4 * real_sz);
        A(&S.field, 2 * (size_t)d.m * real_sz);
        A((void**)&S.adj, npos * 3 * sizeof(double));
        A((void**)&S.apart, (size_t)L.n_bblocks * 4 * sizeof(double));
    }
    const size_t nbins_pad = ((size_t)S.nbins + 32) / 32 * 32 + 32;  // vector scan reads whole 32-bin groups
    A((void**)&S.counts, nbins_pad * sizeof(uint32_t));
    A((void**)&S.bin_start, nbins_pad * sizeof(uint32_t));
    const size_t scan_words = (size_t)(S.nbins + kScanBins - 1) / kScanBins + 1;
    A((void**)&S.scan_status, scan_words * sizeof(unsigned long long));
    A((void**)&S.nbr, ntab * sizeof(int32_t));
    A((void**)&S.nbr_old, ntab * sizeof(int32_t));
    A((void**)&S.nbr_abi, ntab * sizeof(int32_t));
    A((void**)&S.types_abi, npos * sizeof(uint32_t));
    A((void**)&S.qshift, 4 * sizeof(uint32_t));
    A((void**)&S.qshift_next, 4 * sizeof(uint32_t));
    A(&S.spec, 2 * (size_t)d.mz * d.hplane * cplx_sz);
    A(&S.zout, (L.force_ad ? 2 : 4) * (size_t)d.mz * d.hplane * cplx_sz);
    A(&S.fpart, 3 * (size_t)params->order * npos * real_sz);
    A(&S.tw, (size_t)d.ntw() * cplx_sz);
    const bool sampled = (params->flags & TILD_POTENTIAL_SAMPLED) != 0;
    A((void**)&S.utab, (size_t)(d.mx + d.my + d.mz) * sizeof(double));
    if (sampled) A((void**)&S.vtab, (size_t)(d.mx + d.my + d.mz) * sizeof(double));
    A((void**)&S.epart, (size_t)L.n_zblocks * kEpart * sizeof(double));
    A((void**)&S.bpart, (size_t)L.n_bblocks * 4 * sizeof(long long));
    A((void**)&S.noise_part, (size_t)std::max(L.n_bblocks, 2 * d.mz) * 3 * sizeof(long long));
    A((void**)&S.fsum_part, (size_t)2 * d.mz * 3 * sizeof(long long));
    A((void**)&S.flag, sizeof(uint32_t));
    A((void**)&S.eout, 16 * sizeof(double));
    A(&c->staging, npos * 3 * sizeof(double));
    if (measure) {
        *measure = c->ws_used;
        delete c;
        return TILD_OK;
    }
    if (e != hipSuccess) {
        g_create_error = c->ws_base && e == hipErrorOutOfMemory
                             ? "workspace smaller than tild_workspace_bytes"
                             : std::string("device allocation: ") + hipGetErrorString(e);
        tild_destroy(c);
        return e == hipErrorOutOfMemory ? TILD_ENOMEM : TILD_EHIP;
    }
    // Twiddles exp(-2 pi i m / n) in float64, rounded to the working precision.
    std::vector<double> tw;
    for (int a = 0; a < 3; ++a) {
        const int n = a == 0 ? d.mx : (a == 1 ? d.my : d.mz);
        for (int m = 0; m < n; ++m) {
            const double ang = 2.0 * M_PI * (double)m / (double)n;
            tw.push_back(std::cos(ang));
            tw.push_back(-std::sin(ang));
        }
    }
    // two-pass tables: w_n^(l k1) at [l][k1], l < n / r1, k1 < r1 (row pitch r1 + 1, the pad entry 1), for
    // the lengths that use them
    for (const FftPlan* pl : {&L.px, &L.py, &L.pz}) {
        if (!pl->r1) continue;
        const int n = pl->n;
        for (int m = 0; m < n + n / pl->r1; ++m) {
            const int l = m / (pl->r1 + 1), k1 = m % (pl->r1 + 1);
            const double ang = k1 == pl->r1 ? 0.0 : 2.0 * M_PI * (double)((long long)l * k1 % n) / (double)n;
            tw.push_back(std::cos(ang));
            tw.push_back(-std::sin(ang));
        }
    }
    if (tw.size() != 2 * (size_t)d.ntw()) {
        g_create_error = "internal: twiddle table size";
        tild_destroy(c);
        return TILD_EINVAL;
    }
    std::vector<float> twf(tw.begin(), tw.end());
    std::vector<double> ut, vt;
    kernel_tables(*params, d, ut, vt);
    ph.u0 = ut[0] * ut[(size_t)d.mx] * ut[(size_t)(d.mx + d.my)];
    ph.sampled = sampled ? 1 : 0;

    std::vector<uint32_t> types_u((size_t)npos, 0u);
    for (int64_t i = 0; i < n_beads; ++i) types_u[(size_t)i] = (uint32_t)types[i];
    std::vector<uint32_t> zero_bins(((size_t)S.nbins + 32) / 32 * 32 + 32, 0u);
    const uint32_t zeros4[4] = {0, 0, 0, 0};
    auto H2D = [&](void* dst, const void* src, size_t bytes) {
        if (e == hipSuccess && bytes) e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    };
    H2D(S.types_abi, types_u.data(), npos * sizeof(uint32_t));
    H2D(S.nbr_abi, nbr_tab.data(), nbr_tab.size() * sizeof(int32_t));
    H2D(S.counts, zero_bins.data(), zero_bins.size() * sizeof(uint32_t));
    H2D(S.bin_start, zero_bins.data(), zero_bins.size() * sizeof(uint32_t));
    {
        const std::vector<unsigned long long> zero_words(scan_words, 0ull);
        H2D(S.scan_status, zero_words.data(), scan_words * sizeof(unsigned long long));
    }
    H2D(S.qshift, zeros4, sizeof(zeros4));
    H2D(S.qshift_next, zeros4, sizeof(zeros4));
    H2D(S.utab, ut.data(), ut.size() * sizeof(double));
    if (sampled) H2D(S.vtab, vt.data(), vt.size() * sizeof(double));
    else S.vtab = S.utab;
    if (L.precision == 0) H2D(S.tw, twf.data(), twf.size() * sizeof(float));
    else H2D(S.tw, tw.data(), tw.size() * sizeof(double));
    H2D(S.flag, zeros4, sizeof(uint32_t));
    if (ph.gjf && e == hipSuccess) {
        // velocities start at zero; the first placement moves vel_tmp into vel
        e = hipMemset(S.vel, 0, npos * 4 * real_sz);
        if (e == hipSuccess) e = hipMemset(S.vel_tmp, 0, npos * 4 * real_sz);
    }
    if (e == hipSuccess) e = configure_kernel_attributes(L);
    if (e != hipSuccess) {
        g_create_error = std::string("device setup: ") + hipGetErrorString(e);
        tild_destroy(c);
        return TILD_EHIP;
    }
    *out = c;
    return TILD_OK;
}

}  // namespace

TILD_API int tild_create(const tild_params* params, int64_t n_beads, const int32_t* types, int64_t n_bonds,
                         const int32_t* bonds, void* workspace, size_t workspace_bytes, void* hip_stream,
                         tild_ctx** out) {
    return create_impl(params, n_beads, types, n_bonds, bonds, workspace, workspace_bytes, hip_stream, out, nullptr);
}

TILD_API size_t tild_workspace_bytes(const tild_params* params, int64_t n_beads, int64_t n_bonds,
                                     const int32_t* bonds) {
    size_t bytes = 0;
    if (create_impl(params, n_beads, nullptr, n_bonds, bonds, nullptr, 0, nullptr, nullptr, &bytes) != TILD_OK)
        return 0;
    return bytes;
}

TILD_API void tild_destroy(tild_ctx* c) {
    if (!c) return;
    {
        DeviceGuard g(c->device);
        (void)hipStreamSynchronize(c->L.stream);
        for (void* p : c->allocs) (void)hipFree(p);
    }
    delete c;
}

TILD_API const char* tild_last_error(const tild_ctx* c) {
    return c ? c->err.c_str() : g_create_error.c_str();
}

TILD_API int tild_set_positions(tild_ctx* c, const void* xyz, int32_t dtype, int32_t on_device) {
    if (!c) return TILD_EINVAL;
    if ((!xyz && c->S.n > 0) || (dtype != TILD_FP32 && dtype != TILD_FP64))
        return c->fail(TILD_EINVAL, "set_positions: NULL array or bad dtype");
    DeviceGuard g(c->device);
    const size_t esz = dtype == TILD_FP32 ? 4 : 8;
    const size_t bytes = (size_t)c->S.n * 3 * esz;
    const void* src = xyz;
    hipError_t e = hipSuccess;
    if (!on_device && c->S.n > 0) {
        for (int64_t i = 0; i < c->S.n * 3; ++i) {
            const double v = dtype == TILD_FP32 ? (double)((const float*)xyz)[i] : ((const double*)xyz)[i];
            if (!std::isfinite(v)) return c->fail(TILD_EINVAL, "set_positions: non-finite coordinate");
        }
        e = hipMemcpyAsync(c->staging, xyz, bytes, hipMemcpyHostToDevice, c->L.stream);
        src = c->staging;
    }
    // GJF: each bead keeps its velocity; move them to ABI order, the order the placement gives
    if (e == hipSuccess && c->have_pos && c->L.ph.gjf) e = launch_velocities(c->L, c->S, 2, nullptr, 0);
    if (e == hipSuccess) e = launch_place(c->L, c->S, src, dtype);
    if (e == hipSuccess) e = sort_beads(c, c->S.nbr_abi);
    if (e == hipSuccess && !on_device) e = hipStreamSynchronize(c->L.stream);
    if (e != hipSuccess) return c->hip_fail(e, "set_positions");
    c->have_pos = true;
    return TILD_OK;
}

TILD_API int tild_get_positions(tild_ctx* c, void* xyz, int32_t dtype, int32_t on_device) {
    if (!c) return TILD_EINVAL;
    if ((!xyz && c->S.n > 0) || (dtype != TILD_FP32 && dtype != TILD_FP64))
        return c->fail(TILD_EINVAL, "get_positions: NULL array or bad dtype");
    if (!c->have_pos) return c->fail(TILD_ESTATE, "positions were never set");
    DeviceGuard g(c->device);
    const size_t bytes = (size_t)c->S.n * 3 * (dtype == TILD_FP32 ? 4 : 8);
    void* dst = on_device ? xyz : c->staging;
    hipError_t e = launch_get_positions(c->L, c->S, dst, dtype);
    if (e == hipSuccess && !on_device && bytes) e = hipMemcpyAsync(xyz, c->staging, bytes, hipMemcpyDeviceToHost, c->L.stream);
    if (e != hipSuccess) return c->hip_fail(e, "get_positions");
    if (!on_device) return check_flag(c);
    return TILD_OK;
}

TILD_API int tild_set_velocities(tild_ctx* c, const void* v, int32_t dtype, int32_t on_device) {
    if (!c) return TILD_EINVAL;
    if ((!v && c->S.n > 0) || (dtype != TILD_FP32 && dtype != TILD_FP64))
        return c->fail(TILD_EINVAL, "set_velocities: NULL array or bad dtype");
    if (!c->L.ph.gjf) return c->fail(TILD_EINVAL, "set_velocities: the context has no velocities (needs TILD_INTEGRATOR_GJF)");
    if (!c->have_pos) return c->fail(TILD_ESTATE, "positions were never set");
    DeviceGuard g(c->device);
    const size_t bytes = (size_t)c->S.n * 3 * (dtype == TILD_FP32 ? 4 : 8);
    const void* src = v;
    hipError_t e = hipSuccess;
    if (!on_device && c->S.n > 0) {
        for (int64_t i = 0; i < c->S.n * 3; ++i) {
            const double x = dtype == TILD_FP32 ? (double)((const float*)v)[i] : ((const double*)v)[i];
            if (!std::isfinite(x)) return c->fail(TILD_EINVAL, "set_velocities: non-finite value");
        }
        e = hipMemcpyAsync(c->staging, v, bytes, hipMemcpyHostToDevice, c->L.stream);
        src = c->staging;
    }
    if (e == hipSuccess) e = launch_velocities(c->L, c->S, 0, const_cast<void*>(src), dtype);
    if (e == hipSuccess && !on_device) e = hipStreamSynchronize(c->L.stream);
    if (e != hipSuccess) return c->hip_fail(e, "set_velocities");
    return TILD_OK;
}

TILD_API int tild_get_velocities(tild_ctx* c, void* v, int32_t dtype, int32_t on_device) {
    if (!c) return TILD_EINVAL;
    if ((!v && c->S.n > 0) || (dtype != TILD_FP32 && dtype != TILD_FP64))
        return c->fail(TILD_EINVAL, "get_velocities: NULL array or bad dtype");
    if (!c->L.ph.gjf) return c->fail(TILD_EINVAL, "get_velocities: the context has no velocities (needs TILD_INTEGRATOR_GJF)");
    if (!c->have_pos) return c->fail(TILD_ESTATE, "positions were never set");
    DeviceGuard g(c->device);
    const size_t bytes = (size_t)c->S.n * 3 * (dtype == TILD_FP32 ? 4 : 8);
    void* dst = on_device ? v : c->staging;
    hipError_t e = launch_velocities(c->L, c->S, 1, dst, dtype);
    if (e == hipSuccess && !on_device && bytes) e = hipMemcpyAsync(v, c->staging, bytes, hipMemcpyDeviceToHost, c->L.stream);
    if (e != hipSuccess) return c->hip_fail(e, "get_velocities");
    if (!on_device) return check_flag(c);
    return TILD_OK;
}

TILD_API int tild_step(tild_ctx* c, int64_t n_steps) {
    if (!c) return TILD_EINVAL;
    if (n_steps < 0) return c->fail(TILD_EINVAL, "n_steps < 0");
    if (!c->have_pos) return c->fail(TILD_ESTATE, "positions were never set");
    DeviceGuard g(c->device);
    return run_steps(c, n_steps, nullptr);
}

TILD_API int tild_forces(tild_ctx* c, void* out, int32_t dtype, int32_t on_device, uint32_t parts) {
    if (!c) return TILD_EINVAL;
    if ((!out && c->S.n > 0) || (dtype != TILD_FP32 && dtype != TILD_FP64) || parts == 0 || (parts & ~3u))
        return c->fail(TILD_EINVAL, "forces: NULL array, bad dtype or bad parts");
    if (!c->have_pos) return c->fail(TILD_ESTATE, "positions were never set");
    DeviceGuard g(c->device);
    hipError_t e = hipSuccess;
    if (parts & TILD_PART_NONBONDED) e = mesh_forward(c, false);
    void* dst = on_device ? out : c->staging;
    if (e == hipSuccess) e = launch_update(c->L, c->S, 1, (uint64_t)c->step, dst, dtype, parts);
    const size_t bytes = (size_t)c->S.n * 3 * (dtype == TILD_FP32 ? 4 : 8);
    if (e == hipSuccess && !on_device && bytes) e = hipMemcpyAsync(out, c->staging, bytes, hipMemcpyDeviceToHost, c->L.stream);
    if (e != hipSuccess) return c->hip_fail(e, "forces");
    if (!on_device) return check_flag(c);
    return TILD_OK;
}

TILD_API int tild_interaction_forces(tild_ctx* c, double chi, double kappa, int32_t with_charges, void* out,
                                    int32_t dtype, int32_t on_device) {
    if (!c) return TILD_EINVAL;
    if ((!out && c->S.n > 0) || (dtype != TILD_FP32 && dtype != TILD_FP64) || !std::isfinite(chi) ||
        !std::isfinite(kappa))
        return c->fail(TILD_EINVAL, "interaction_forces: NULL array, bad dtype or non-finite chi/kappa");
    if (!c->have_pos) return c->fail(TILD_ESTATE, "positions were never set");
    DeviceGuard g(c->device);
    // the kernels take the physics by value: a modified copy needs no table change
    Launch L = c->L;
    L.ph.chi = chi;
    L.ph.kappa = kappa;
    if (!with_charges) L.ph.elec = 0;
    hipError_t e = launch_spread_xy(L, c->S);
    if (e == hipSuccess) e = launch_z_kmul(L, c->S, false);
    if (e == hipSuccess) e = launch_xy_c2r(L, c->S);
    void* dst = on_device ? out : c->staging;
    if (e == hipSuccess) e = launch_update(L, c->S, 1, (uint64_t)c->step, dst, dtype, TILD_PART_NONBONDED);
    const size_t bytes = (size_t)c->S.n * 3 * (dtype == TILD_FP32 ? 4 : 8);
    if (e == hipSuccess && !on_device && bytes) e = hipMemcpyAsync(out, c->staging, bytes, hipMemcpyDeviceToHost, c->L.stream);
    if (e != hipSuccess) return c->hip_fail(e, "interaction_forces");
    if (!on_device) return check_flag(c);
    return TILD_OK;
}

TILD_API int tild_energy(tild_ctx* c, double out[8]) {
    if (!c) return TILD_EINVAL;
    if (!out) return c->fail(TILD_EINVAL, "energy: out is NULL");
    if (!c->have_pos) return c->fail(TILD_ESTATE, "positions were never set");
    DeviceGuard g(c->device);
    hipError_t e = mesh_forward(c, true);
    if (e == hipSuccess) e = launch_bond_energy(c->L, c->S);
    if (e == hipSuccess) e = launch_reduce_energy(c->L, c->S);
    if (e == hipSuccess) e = hipMemcpyAsync(out, c->S.eout, 8 * sizeof(double), hipMemcpyDeviceToHost, c->L.stream);
    if (e != hipSuccess) return c->hip_fail(e, "energy");
    return check_flag(c);
}

TILD_API int tild_counts(tild_ctx* c, void* out, int32_t on_device) {
    if (!c) return TILD_EINVAL;
    if (!out) return c->fail(TILD_EINVAL, "counts: out is NULL");
    if (!c->have_pos) return c->fail(TILD_ESTATE, "positions were never set");
    DeviceGuard g(c->device);
    const size_t bytes = 2 * (size_t)c->L.d.m * (c->L.precision == 0 ? 4 : 8);
    void* dst = on_device ? out : c->S.zout;  // zout holds at least 2 M reals
    hipError_t e = launch_counts(c->L, c->S, dst);
    if (e == hipSuccess && !on_device) e = hipMemcpyAsync(out, c->S.zout, bytes, hipMemcpyDeviceToHost, c->L.stream);
    if (e != hipSuccess) return c->hip_fail(e, "counts");
    if (!on_device) return check_flag(c);
    return TILD_OK;
}

TILD_API int tild_field_forces(tild_ctx* c, const void* field, void* out, int32_t dtype, int32_t on_device) {
    if (!c) return TILD_EINVAL;
    if (!field || (!out && c->S.n > 0) || (dtype != TILD_FP32 && dtype != TILD_FP64))
        return c->fail(TILD_EINVAL, "field_forces: NULL array or bad dtype");
    if (c->L.order < 2) return c->fail(TILD_EINVAL, "field_forces: needs order >= 2");
    if (!c->have_pos) return c->fail(TILD_ESTATE, "positions were never set");
    DeviceGuard g(c->device);
    const size_t gbytes = 2 * (size_t)c->L.d.m * (c->L.precision == 0 ? 4 : 8);
    const size_t bytes = (size_t)c->S.n * 3 * (dtype == TILD_FP32 ? 4 : 8);
    hipError_t e = hipSuccess;
    const void* src = field;
    if (!on_device) {
        e = hipMemcpyAsync(c->S.zout, field, gbytes, hipMemcpyHostToDevice, c->L.stream);
        src = c->S.zout;
    }
    void* dst = on_device ? out : c->staging;
    if (e == hipSuccess) e = launch_field_forces(c->L, c->S, src, dst, dtype);
    if (e == hipSuccess && !on_device && bytes) e = hipMemcpyAsync(out, c->staging, bytes, hipMemcpyDeviceToHost, c->L.stream);
    if (e != hipSuccess) return c->hip_fail(e, "field_forces");
    if (!on_device) return check_flag(c);
    return TILD_OK;
}

TILD_API int tild_hvp(tild_ctx* c, const void* v, void* out, int32_t dtype, int32_t on_device) {
    if (!c) return TILD_EINVAL;
    if (((!v || !out) && c->S.n > 0) || (dtype != TILD_FP32 && dtype != TILD_FP64))
        return c->fail(TILD_EINVAL, "hvp: NULL array or bad dtype");
    if (c->L.order < 3) return c->fail(TILD_EINVAL, "hvp: needs order >= 3");
    if (!c->have_pos) return c->fail(TILD_ESTATE, "positions were never set");
    DeviceGuard g(c->device);
    const size_t bytes = (size_t)c->S.n * 3 * (dtype == TILD_FP32 ? 4 : 8);
    hipError_t e = hipSuccess;
    const void* src = v;
    if (!on_device && c->S.n > 0) {
        for (int64_t i = 0; i < c->S.n * 3; ++i) {
            const double x = dtype == TILD_FP32 ? (double)((const float*)v)[i] : ((const double*)v)[i];
            if (!std::isfinite(x)) return c->fail(TILD_EINVAL, "hvp: non-finite direction");
        }
        e = hipMemcpyAsync(c->staging, v, bytes, hipMemcpyHostToDevice, c->L.stream);
        src = c->staging;
    }
    // the result overwrites the staging copy of v only after v was read (stream order)
    void* dst = on_device ? out : c->staging;
    if (e == hipSuccess) e = launch_hvp(c->L, c->S, src, dst, dtype);
    if (e == hipSuccess && !on_device && bytes) e = hipMemcpyAsync(out, c->staging, bytes, hipMemcpyDeviceToHost, c->L.stream);
    if (e != hipSuccess) return c->hip_fail(e, "hvp");
    if (!on_device) return check_flag(c);
    return TILD_OK;
}

namespace {

// out (device, dtype) = (dF/dx)^T lam (device, dtype) at the current positions, F the context's force
// (non-bonded route and bonds): the ik route's transposed Jacobian, or -H lam on the exact-gradient route.
hipError_t force_vjp(tild_ctx* c, const void* lam, void* out, int dtype) {
    if (!c->L.force_ad) return launch_force_vjp_ik(c->L, c->S, lam, out, dtype);
    hipError_t e = launch_hvp(c->L, c->S, lam, out, dtype);
    if (e == hipSuccess) e = launch_adjoint_vectors(c->L, c->S, AdjointOp::kScale, out, nullptr, dtype, -1.0, nullptr);
    return e;
}

// Non-bonded forces of the interaction (chi, kappa), no charges, on the context's route, to out (device,
// float64, ABI order).
hipError_t pure_interaction_forces(tild_ctx* c, double chi, double kappa, double* out) {
    Launch L = c->L;
    L.ph.chi = chi;
    L.ph.kappa = kappa;
    L.ph.elec = 0;
    hipError_t e = launch_spread_xy(L, c->S);
    if (e == hipSuccess) e = launch_z_kmul(L, c->S, false);
    if (e == hipSuccess) e = launch_xy_c2r(L, c->S);
    if (e == hipSuccess) e = launch_update(L, c->S, 1, (uint64_t)c->step, out, TILD_FP64, TILD_PART_NONBONDED);
    return e;
}

}  // namespace

TILD_API int tild_force_vjp(tild_ctx* c, const void* lam, void* out, int32_t dtype, int32_t on_device) {
    if (!c) return TILD_EINVAL;
    if (((!lam || !out) && c->S.n > 0) || (dtype != TILD_FP32 && dtype != TILD_FP64))
        return c->fail(TILD_EINVAL, "force_vjp: NULL array or bad dtype");
    if (c->L.order < (c->L.force_ad ? 3 : 2))
        return c->fail(TILD_EINVAL, "force_vjp: needs order >= 2 (ik route) or >= 3 (exact-gradient route)");
    if (!c->have_pos) return c->fail(TILD_ESTATE, "positions were never set");
    DeviceGuard g(c->device);
    const size_t bytes = (size_t)c->S.n * 3 * (dtype == TILD_FP32 ? 4 : 8);
    hipError_t e = hipSuccess;
    const void* src = lam;
    if (!on_device && c->S.n > 0) {
        for (int64_t i = 0; i < c->S.n * 3; ++i) {
            const double x = dtype == TILD_FP32 ? (double)((const float*)lam)[i] : ((const double*)lam)[i];
            if (!std::isfinite(x)) return c->fail(TILD_EINVAL, "force_vjp: non-finite vector");
        }
        e = hipMemcpyAsync(c->staging, lam, bytes, hipMemcpyHostToDevice, c->L.stream);
        src = c->staging;
    }
    void* dst = on_device ? out : c->staging;  // lam is read before the result is written (stream order)
    if (e == hipSuccess && c->S.n > 0) e = force_vjp(c, src, dst, dtype);
    if (e == hipSuccess && !on_device && bytes) e = hipMemcpyAsync(out, c->staging, bytes, hipMemcpyDeviceToHost, c->L.stream);
    if (e != hipSuccess) return c->hip_fail(e, "force_vjp");
    if (!on_device) return check_flag(c);
    return TILD_OK;
}

TILD_API int tild_adjoint_step(tild_ctx* c, double* lam, double* dtheta) {
    if (!c) return TILD_EINVAL;
    if ((!lam && c->S.n > 0) || !dtheta) return c->fail(TILD_EINVAL, "adjoint_step: NULL array");
    if (c->L.order < (c->L.force_ad ? 3 : 2))
        return c->fail(TILD_EINVAL, "adjoint_step: needs order >= 2 (ik route) or >= 3 (exact-gradient route)");
    if (c->L.ph.gjf) return c->fail(TILD_EINVAL, "adjoint_step: Euler-Maruyama contexts only");
    if (!c->have_pos) return c->fail(TILD_ESTATE, "positions were never set");
    if (c->S.n == 0) return TILD_OK;
    DeviceGuard g(c->device);
    const double mu = c->p.dt / c->p.gamma;
    double* pl = static_cast<double*>(c->staging);
    double* mean = c->S.eout + 12;  // eout[12..14]: the mean of lambda
    hipError_t e = hipSuccess;
    // Pr lambda: lambda minus its mean over the beads with centre-of-mass correction
    if (c->L.ph.com_correct)
        e = launch_adjoint_vectors(c->L, c->S, AdjointOp::kMean, lam, nullptr, TILD_FP64, 0.0, mean);
    if (e == hipSuccess)
        e = launch_adjoint_vectors(c->L, c->S, AdjointOp::kProject, lam, pl, TILD_FP64, 0.0,
                                   c->L.ph.com_correct ? mean : nullptr);
    // dL/dtheta += mu (Pr lambda) . dF/dtheta, dF/dchi and dF/dkappa the forces of the pure interactions
    if (e == hipSuccess) e = pure_interaction_forces(c, 1.0, 0.0, c->S.adj);
    if (e == hipSuccess) e = launch_adjoint_vectors(c->L, c->S, AdjointOp::kDotAdd, pl, c->S.adj, TILD_FP64, mu, dtheta);
    if (e == hipSuccess) e = pure_interaction_forces(c, 0.0, 1.0, c->S.adj);
    if (e == hipSuccess)
        e = launch_adjoint_vectors(c->L, c->S, AdjointOp::kDotAdd, pl, c->S.adj, TILD_FP64, mu, dtheta + 1);
    // lambda += mu J^T Pr lambda
    if (e == hipSuccess) e = force_vjp(c, pl, c->S.adj, TILD_FP64);
    if (e == hipSuccess) e = launch_adjoint_vectors(c->L, c->S, AdjointOp::kAxpy, lam, c->S.adj, TILD_FP64, mu, nullptr);
    if (e != hipSuccess) return c->hip_fail(e, "adjoint_step");
    return TILD_OK;
}

TILD_API int tild_set_interaction(tild_ctx* c, double chi, double kappa, double smear_a) {
    if (!c) return TILD_EINVAL;
    if (!std::isfinite(chi) || !std::isfinite(kappa) || !std::isfinite(smear_a) || smear_a < 0.0)
        return c->fail(TILD_EINVAL, "set_interaction: chi, kappa must be finite and smear_a finite and >= 0");
    if ((c->p.flags & TILD_POTENTIAL_SAMPLED) && !(smear_a > 0.0))
        return c->fail(TILD_EINVAL, "set_interaction: TILD_POTENTIAL_SAMPLED needs smear_a > 0");
    DeviceGuard g(c->device);
    // the tables may still be read by queued work
    hipError_t e = hipStreamSynchronize(c->L.stream);
    tild_params p = c->p;
    p.chi = chi;
    p.kappa = kappa;
    p.smear_a = smear_a;
    std::vector<double> ut, vt;
    kernel_tables(p, c->L.d, ut, vt);
    if (e == hipSuccess) e = hipMemcpy(c->S.utab, ut.data(), ut.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess && c->S.vtab != c->S.utab)
        e = hipMemcpy(c->S.vtab, vt.data(), vt.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return c->hip_fail(e, "set_interaction");
    c->p = p;
    Phys& ph = c->L.ph;
    ph.chi = chi;
    ph.kappa = kappa;
    ph.a2 = smear_a * smear_a;
    ph.u0 = ut[0] * ut[(size_t)c->L.d.mx] * ut[(size_t)(c->L.d.mx + c->L.d.my)];
    return TILD_OK;
}

TILD_API int tild_energy_grad(tild_ctx* c, double out[4], void* grad_x, int32_t dtype, int32_t on_device) {
    if (!c) return TILD_EINVAL;
    if (!out || (dtype != TILD_FP32 && dtype != TILD_FP64))
        return c->fail(TILD_EINVAL, "energy_grad: NULL out or bad dtype");
    if (!c->have_pos) return c->fail(TILD_ESTATE, "positions were never set");
    if (grad_x && c->L.order < 2) return c->fail(TILD_EINVAL, "energy_grad: dE/dx needs order >= 2");
    DeviceGuard g(c->device);
    hipError_t e = launch_spread_xy(c->L, c->S);
    if (e == hipSuccess) e = launch_z_kmul(c->L, c->S, grad_x == nullptr, true);
    if (e == hipSuccess) e = launch_bond_energy(c->L, c->S);
    if (e == hipSuccess) e = launch_reduce_energy(c->L, c->S);
    double eo[16];
    if (e == hipSuccess) e = hipMemcpyAsync(eo, c->S.eout, sizeof(eo), hipMemcpyDeviceToHost, c->L.stream);
    const size_t bytes = (size_t)c->S.n * 3 * (dtype == TILD_FP32 ? 4 : 8);
    if (grad_x) {
        // dE/dx = -(F_nb by the exact gradient + F_bond), whatever the context's route
        if (e == hipSuccess) e = launch_xy_c2r(c->L, c->S, 1);
        void* dst = on_device ? grad_x : c->staging;
        if (e == hipSuccess) e = launch_update(c->L, c->S, 1, (uint64_t)c->step, dst, dtype, TILD_PART_TOTAL, -1.0);
        if (e == hipSuccess && !on_device && bytes)
            e = hipMemcpyAsync(grad_x, c->staging, bytes, hipMemcpyDeviceToHost, c->L.stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->L.stream);
    if (e != hipSuccess) return c->hip_fail(e, "energy_grad");
    out[0] = eo[3];
    out[1] = eo[8];
    out[2] = eo[9];
    out[3] = eo[10];
    return check_flag(c);
}

TILD_API int64_t tild_step_count(const tild_ctx* c) { return c ? c->step : -1; }

TILD_API int tild_set_step_count(tild_ctx* c, int64_t step) {
    if (!c) return TILD_EINVAL;
    if (step < 0) return c->fail(TILD_EINVAL, "step < 0");
    c->step = step;
    return TILD_OK;
}

TILD_API int tild_synchronize(tild_ctx* c) {
    if (!c) return TILD_EINVAL;
    DeviceGuard g(c->device);
    return check_flag(c);
}

TILD_API int tild_profile_steps(tild_ctx* c, int64_t n_steps, double* kernel_ms, int32_t* launches_per_step,
                                int32_t n_slots) {
    if (!c) return TILD_EINVAL;
    if (n_steps < 1 || !kernel_ms || n_slots < 1 || n_slots > kNumSlots)
        return c->fail(TILD_EINVAL, "profile_steps: bad arguments");
    if (!c->have_pos) return c->fail(TILD_ESTATE, "positions were never set");
    DeviceGuard g(c->device);
    std::vector<hipEvent_t> ev((size_t)n_steps * kNumSlots * 2, nullptr);
    hipError_t e = hipSuccess;
    for (auto& x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    int rc = TILD_OK;
    if (e == hipSuccess) rc = run_steps(c, n_steps, &ev);
    if (e == hipSuccess && rc == TILD_OK) e = hipStreamSynchronize(c->L.stream);
    std::vector<double> sum(kNumSlots, 0.0);
    for (int64_t s = 0; e == hipSuccess && rc == TILD_OK && s < n_steps; ++s)
        for (int k = 0; k < kNumSlots; ++k) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[(size_t)(s * kNumSlots + k) * 2], ev[(size_t)(s * kNumSlots + k) * 2 + 1]);
            if (e != hipSuccess) break;
            sum[(size_t)k] += ms;
        }
    for (auto& x : ev)
        if (x) (void)hipEventDestroy(x);
    if (rc != TILD_OK) return rc;
    if (e != hipSuccess) return c->hip_fail(e, "profile_steps");
    for (int k = 0; k < n_slots; ++k) {
        kernel_ms[k] = sum[(size_t)k] / (double)n_steps;
        if (launches_per_step) launches_per_step[k] = (k == kUpdate && c->L.force_ad) ? 2 : 1;
    }
    return check_flag(c);
}

TILD_API const char* tild_kernel_name(int32_t slot) {
    if (slot < 0 || slot >= kNumSlots) return nullptr;
    return kSlotNames[slot];
}

TILD_API int tild_stream_copy(void* dst, const void* src, size_t bytes, int32_t iters, void* hip_stream,
                              double* ms_per_copy) {
    if (!dst || !src || bytes == 0 || bytes % 16 || iters < 1 || !ms_per_copy) {
        g_create_error = "stream_copy: bad arguments";
        return TILD_EINVAL;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipEventRecord(a, s);
    for (int i = 0; e == hipSuccess && i < iters; ++i) e = launch_stream_copy(dst, src, bytes, s);
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) {
        g_create_error = std::string("stream_copy: ") + hipGetErrorString(e);
        return TILD_EHIP;
    }
    *ms_per_copy = ms / iters;
    return TILD_OK;
}

// ---------------------------------------------------------------- batches

namespace {

// Member indices ordered by grid size (then bead count), largest first.
std::vector<int32_t> members_by_size(tild_ctx* const* ctxs, int32_t n_ctx) {
    std::vector<int32_t> order((size_t)n_ctx);
    for (int32_t r = 0; r < n_ctx; ++r) order[(size_t)r] = r;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const tild_ctx *ca = ctxs[a], *cb = ctxs[b];
        if (ca->L.d.m != cb->L.d.m) return ca->L.d.m > cb->L.d.m;
        return ca->S.n > cb->S.n;
    });
    return order;
}

}  // namespace

struct tild_batch {
    std::vector<tild_ctx*> ctx;
    hipStream_t stream = nullptr;
    int device = 0;
    Launch L{};
    RepDesc* h_desc = nullptr;  // pinned host copy of the descriptors
    RepDesc* d_desc = nullptr;
    uint32_t* maps = nullptr;
    unsigned long long* status = nullptr;  // every member's scan status words, then the ticket
    std::vector<size_t> status_off;
    BatchMaps B{};
    size_t lds_plane = 0, lds_z = 0;
    std::vector<hipEvent_t> member_ev;
    hipEvent_t copy_ev = nullptr, done_ev = nullptr;
    bool copy_pending = false;
    // steps replayed from a captured graph: n_steps launches of every batched kernel, captured on a
    // private stream the first time a call asks for that many steps
    bool use_graph = true;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t exec_steps = 0;
    int exec_block = 0;  // plane_block the graph was captured with
    // column block of the batched k-space pass: 0 = each member's own (its single-context choice), else this
    // many columns for every member; zc / nzb: the columns per block and blocks each member uses
    int z_cols = 0;
    std::vector<int> zc, nzb;
    std::string err;

    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
        exec_steps = 0;
    }

    int fail(int code, const std::string& msg) {
        err = msg;
        return code;
    }
    int hip_fail(hipError_t e, const char* what) {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return TILD_EHIP;
    }
};

TILD_API void tild_batch_destroy(tild_batch* b) {
    if (!b) return;
    {
        DeviceGuard g(b->device);
        (void)hipStreamSynchronize(b->stream);
        if (b->h_desc) (void)hipHostFree(b->h_desc);
        if (b->d_desc) (void)hipFree(b->d_desc);
        if (b->maps) (void)hipFree(b->maps);
        if (b->status) (void)hipFree(b->status);
        for (hipEvent_t e : b->member_ev)
            if (e) (void)hipEventDestroy(e);
        if (b->copy_ev) (void)hipEventDestroy(b->copy_ev);
        if (b->done_ev) (void)hipEventDestroy(b->done_ev);
        b->drop_graph();
        if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    }
    delete b;
}

namespace {

// (Re)build a batch's unit maps, scan status words and LDS sizes for k-space column blocks of z_cols
// columns (0: each member's own).  Member by member, the largest grids first (their planes and column
// blocks take longest, so the last round of workgroups holds the short ones); every member's scan keeps
// its own status words.  hipErrorInvalidValue if a member's column block would not fit the LDS.
hipError_t build_batch_maps(tild_batch* b, int z_cols) {
    const int32_t n_ctx = (int32_t)b->ctx.size();
    std::vector<uint32_t> plane, c2r, zcol, bead, tile, plane_small, c2r_small;
    std::vector<int> zc((size_t)n_ctx), nzb((size_t)n_ctx);
    std::vector<size_t> status_off((size_t)n_ctx, 0);
    size_t nstatus = 0, lds_plane = 0, lds_z = 0, lds_small = 0;
    for (const int32_t r : members_by_size(b->ctx.data(), n_ctx)) {
        const tild_ctx* c = b->ctx[(size_t)r];
        const Dims& d = c->L.d;
        Launch Lz = c->L;
        if (z_cols > 0) Lz.z_cols = (int)std::min<long long>(z_cols, d.hplane);
        zc[(size_t)r] = Lz.z_cols;
        nzb[(size_t)r] = (int)((d.hplane + Lz.z_cols - 1) / Lz.z_cols);
        const uint32_t hi = (uint32_t)r << 16;
        // small planes (LDS for eight workgroups per CU) go to a launch of their own with fewer threads per
        // workgroup
        const size_t lds = plane_lds_bytes(c->L);
        const bool small = lds <= kSmallPlaneLds;
        for (int u = 0; u < 2 * d.mz; ++u) (small ? plane_small : plane).push_back(hi | (uint32_t)u);
        for (int u = 0; u < 6 * d.mz; ++u) (small ? c2r_small : c2r).push_back(hi | (uint32_t)u);
        for (int u = 0; u < nzb[(size_t)r]; ++u) zcol.push_back(hi | (uint32_t)u);
        for (long long u = 0; u < (c->S.n + 255) / 256; ++u) bead.push_back(hi | (uint32_t)u);
        const int ntiles = (c->S.nbins + kScanBins - 1) / kScanBins;
        for (int u = 0; u < ntiles; ++u) tile.push_back(hi | (uint32_t)u);
        status_off[(size_t)r] = nstatus;
        nstatus += (size_t)ntiles;
        if (small) lds_small = std::max(lds_small, lds);
        else lds_plane = std::max(lds_plane, lds);
        lds_z = std::max(lds_z, z_lds_bytes(Lz));
        if (nzb[(size_t)r] > 65535) return hipErrorInvalidValue;
    }
    const int n_plane_small = (int)plane_small.size(), n_c2r_small = (int)c2r_small.size();
    int deg_all = b->ctx[0]->S.deg;
    for (const tild_ctx* c : b->ctx)
        if (c->S.deg != deg_all) deg_all = 0;
    plane.insert(plane.end(), plane_small.begin(), plane_small.end());
    c2r.insert(c2r.end(), c2r_small.begin(), c2r_small.end());
    if (lds_z > 160 * 1024) return hipErrorInvalidValue;
    const size_t nmap = plane.size() + c2r.size() + zcol.size() + bead.size() + tile.size();
    std::vector<uint32_t> all;
    all.reserve(nmap);
    for (const auto* v : {&plane, &c2r, &zcol, &bead, &tile}) all.insert(all.end(), v->begin(), v->end());
    // the old maps may still be read by queued work, and the graph captured over them is dropped
    hipError_t e = hipStreamSynchronize(b->stream);
    b->drop_graph();
    if (b->maps) (void)hipFree(b->maps);
    if (b->status) (void)hipFree(b->status);
    b->maps = nullptr;
    b->status = nullptr;
    if (e == hipSuccess) e = hipMalloc((void**)&b->maps, nmap * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemcpy(b->maps, all.data(), nmap * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc((void**)&b->status, (nstatus + 1) * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemset(b->status, 0, (nstatus + 1) * sizeof(unsigned long long));
    if (e == hipSuccess) e = configure_batch_attributes(b->L, lds_plane, lds_z);
    if (e != hipSuccess) return e;
    BatchMaps& B = b->B;
    B.plane = b->maps;
    B.c2r = B.plane + plane.size();
    B.zcol = B.c2r + c2r.size();
    B.bead = B.zcol + zcol.size();
    B.tile = B.bead + bead.size();
    B.n_plane = (int)plane.size();
    B.n_c2r = (int)c2r.size();
    B.n_plane_small = n_plane_small;
    B.n_c2r_small = n_c2r_small;
    B.lds_small = lds_small;
    B.deg = deg_all >= 1 && deg_all <= 4 ? deg_all : 0;
    B.n_zcol = (int)zcol.size();
    B.n_bead = (int)bead.size();
    B.n_tile = (int)tile.size();
    B.ticket = b->status + nstatus;
    b->status_off = status_off;
    b->zc = zc;
    b->nzb = nzb;
    b->z_cols = z_cols;
    b->lds_plane = lds_plane;
    b->lds_z = lds_z;
    return hipSuccess;
}

}  // namespace

TILD_API int tild_batch_create(tild_ctx* const* ctxs, int32_t n_ctx, void* hip_stream, tild_batch** out) {
    if (!out) return TILD_EINVAL;
    *out = nullptr;
    auto bad = [&](const std::string& why) {
        g_create_error = "batch: " + why;
        return TILD_EINVAL;
    };
    if (!ctxs || n_ctx < 1 || n_ctx > 65535) return bad("needs 1..65535 contexts");
    const tild_ctx* c0 = ctxs[0];
    if (!c0) return bad("NULL context");
    for (int32_t i = 0; i < n_ctx; ++i) {
        const tild_ctx* c = ctxs[i];
        if (!c) return bad("NULL context");
        for (int32_t k = 0; k < i; ++k)
            if (ctxs[k] == c) return bad("a context appears twice");
        if (c->device != c0->device) return bad("contexts on different devices");
        if (c->L.precision != c0->L.precision || c->L.order != c0->L.order || c->p.flags != c0->p.flags ||
            c->L.ph.elec != c0->L.ph.elec)
            return bad("contexts differ in precision, order, flags or the presence of charges");
        if (c->L.force_ad || c->L.ph.gjf) return bad("batched steps use the ik route and Euler-Maruyama");
        if ((c->S.n + 255) / 256 > 65535) return bad("a member has more than 16,776,960 beads");
    }
    tild_batch* b = new (std::nothrow) tild_batch();
    if (!b) {
        g_create_error = "out of host memory";
        return TILD_ENOMEM;
    }
    b->device = c0->device;
    b->stream = (hipStream_t)hip_stream;
    b->ctx.assign(ctxs, ctxs + n_ctx);
    b->L = c0->L;
    b->L.stream = b->stream;
    DeviceGuard g(b->device);
    hipError_t e = build_batch_maps(b, 0);
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_desc, (size_t)n_ctx * sizeof(RepDesc));
    if (e == hipSuccess) e = hipHostMalloc((void**)&b->h_desc, (size_t)n_ctx * sizeof(RepDesc), hipHostMallocDefault);
    b->member_ev.assign((size_t)n_ctx, nullptr);
    for (int32_t r = 0; e == hipSuccess && r < n_ctx; ++r)
        e = hipEventCreateWithFlags(&b->member_ev[(size_t)r], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->copy_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        g_create_error = std::string("batch: device setup: ") + hipGetErrorString(e);
        tild_batch_destroy(b);
        return TILD_EHIP;
    }
    BatchMaps& B = b->B;
    B.reps = b->d_desc;
    // measured on MI355X with 64 replicas of 32^2..80^2 planes: 256-thread plane workgroups are 13 %
    // faster than 512 (several small planes per CU); larger planes keep 512
    int max_plane = 0;
    for (const tild_ctx* c : b->ctx) max_plane = std::max(max_plane, c->L.d.mx * c->L.d.my);
    B.plane_block = max_plane <= 96 * 96 ? 256 : 512;
    *out = b;
    return TILD_OK;
}

TILD_API int tild_batch_step(tild_batch* b, int64_t n_steps) {
    if (!b) return TILD_EINVAL;
    if (n_steps < 0 || n_steps > 0x7fffffffLL) return b->fail(TILD_EINVAL, "n_steps must be in [0, 2^31)");
    for (tild_ctx* c : b->ctx)
        if (!c->have_pos) return b->fail(TILD_ESTATE, "a member's positions were never set");
    if (n_steps == 0) return TILD_OK;
    DeviceGuard g(b->device);
    hipError_t e = hipSuccess;
    // the batch's stream waits for the work already queued on every member's stream
    for (size_t r = 0; e == hipSuccess && r < b->ctx.size(); ++r) {
        e = hipEventRecord(b->member_ev[r], b->ctx[r]->L.stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->member_ev[r], 0);
    }
    // the previous call's descriptor upload must have left the pinned buffer
    if (e == hipSuccess && b->copy_pending) e = hipEventSynchronize(b->copy_ev);
    for (size_t r = 0; e == hipSuccess && r < b->ctx.size(); ++r) {
        const tild_ctx* c = b->ctx[r];
        RepDesc& R = b->h_desc[r];
        R.d = c->L.d;
        R.px = c->L.px;
        R.py = c->L.py;
        R.pz = c->L.pz;
        R.ph = c->L.ph;
        R.S = c->S;
        R.S.scan_status = b->status + b->status_off[r];
        R.ntiles = (c->S.nbins + kScanBins - 1) / kScanBins;
        R.step0 = (uint64_t)c->step;
        R.z_cols = b->zc[r];
        R.n_zblocks = b->nzb[r];
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_desc, b->h_desc, b->ctx.size() * sizeof(RepDesc), hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->copy_ev, b->stream);
    if (e == hipSuccess) b->copy_pending = true;
    if (e == hipSuccess && b->use_graph) {
        if (!b->exec || b->exec_steps != n_steps || b->exec_block != b->B.plane_block) {
            // the kernels read every member's state from the descriptors uploaded above, so the graph
            // of n_steps steps serves every later call of that many steps
            b->drop_graph();
            Launch Lc = b->L;
            Lc.stream = b->cap_stream;
            hipGraph_t graph = nullptr;
            e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) e = launch_batch_noise(Lc, b->B);
            for (int64_t s = 0; e == hipSuccess && s < n_steps; ++s)
                e = launch_batch_step(Lc, b->B, (int)s, b->lds_plane, b->lds_z);
            const hipError_t ec = hipStreamEndCapture(b->cap_stream, &graph);
            if (e == hipSuccess) e = ec;
            if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (e == hipSuccess) {
                b->exec_steps = n_steps;
                b->exec_block = b->B.plane_block;
            } else {
                b->drop_graph();
            }
        }
        if (e == hipSuccess) e = hipGraphLaunch(b->exec, b->stream);
    } else {
        if (e == hipSuccess) e = launch_batch_noise(b->L, b->B);
        for (int64_t s = 0; e == hipSuccess && s < n_steps; ++s)
            e = launch_batch_step(b->L, b->B, (int)s, b->lds_plane, b->lds_z);
    }
    if (e != hipSuccess) {
        for (tild_ctx* c : b->ctx) c->noise_ready = -1;
        return b->hip_fail(e, "batch step");
    }
    // the members' pointer pairs swap once per step; their step counters advance, and the last scatter left
    // the noise sums of the step they reach
    for (tild_ctx* c : b->ctx) {
        if (n_steps & 1) {
            std::swap(c->S.qshift, c->S.qshift_next);
            std::swap(c->S.nbr, c->S.nbr_old);
        }
        c->step += n_steps;
        c->noise_ready = c->step;
    }
    // later work on a member's stream waits for the batch
    e = hipEventRecord(b->done_ev, b->stream);
    for (size_t r = 0; e == hipSuccess && r < b->ctx.size(); ++r) e = hipStreamWaitEvent(b->ctx[r]->L.stream, b->done_ev, 0);
    if (e != hipSuccess) return b->hip_fail(e, "batch step");
    return TILD_OK;
}

TILD_API int tild_batch_autotune(tild_batch* b, int32_t trial_steps, int32_t* plane_block, int32_t* z_cols,
                                int32_t* graph) {
    if (!b) return TILD_EINVAL;
    if (trial_steps < 1 || trial_steps > 1000) return b->fail(TILD_EINVAL, "autotune: trial_steps must be in [1, 1000]");
    for (tild_ctx* c : b->ctx)
        if (!c->have_pos) return b->fail(TILD_ESTATE, "a member's positions were never set");
    DeviceGuard g(b->device);
    // snapshot: every member's positions (ABI order, float64) and step counter
    std::vector<size_t> off;
    size_t total = 0;
    for (tild_ctx* c : b->ctx) {
        off.push_back(total);
        total += (size_t)c->S.n * 3;
    }
    double* snap = nullptr;
    hipError_t e = hipMalloc((void**)&snap, std::max<size_t>(total, 1) * sizeof(double));
    if (e != hipSuccess) return b->fail(TILD_ENOMEM, "autotune: no device memory for the snapshot");
    std::vector<int64_t> step0;
    for (size_t r = 0; e == hipSuccess && r < b->ctx.size(); ++r) {
        tild_ctx* c = b->ctx[r];
        step0.push_back(c->step);
        e = launch_get_positions(c->L, c->S, snap + off[r], 1);  // on the member's own stream
    }
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&t0);
    if (e == hipSuccess) e = hipEventCreate(&t1);
    const int keep_block = b->B.plane_block, keep_z = b->z_cols;
    const bool keep_graph = b->use_graph;
    int rc = TILD_OK;
    // one trial: trial_steps batched steps, timed on the batch's stream, the state restored afterwards
    auto trial = [&](int block, bool use_graph) -> float {
        b->B.plane_block = block;
        b->use_graph = use_graph;
        float ms = 1e30f;
        for (size_t r = 0; e == hipSuccess && r < b->ctx.size(); ++r) {
            e = hipEventRecord(b->member_ev[r], b->ctx[r]->L.stream);
            if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->member_ev[r], 0);
        }
        if (e == hipSuccess) e = hipEventRecord(t0, b->stream);
        if (e == hipSuccess && rc == TILD_OK) rc = tild_batch_step(b, trial_steps);
        if (rc == TILD_OK && e == hipSuccess) e = hipEventRecord(t1, b->stream);
        if (rc == TILD_OK && e == hipSuccess) e = hipEventSynchronize(t1);
        if (rc == TILD_OK && e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
        for (size_t r = 0; rc == TILD_OK && r < b->ctx.size(); ++r) {
            rc = tild_set_positions(b->ctx[r], snap + off[r], TILD_FP64, 1);
            b->ctx[r]->step = step0[r];
            b->ctx[r]->noise_ready = -1;
        }
        return ms;
    };
    // plane-workgroup sizes with eager launches, each twice, alternating; then the faster one replayed
    // from a captured graph (one untimed call captures it)
    const int cand[2] = {256, 512};
    float best_ms[2] = {1e30f, 1e30f};
    for (int rep = 0; rep < 4 && e == hipSuccess && rc == TILD_OK; ++rep)
        best_ms[rep & 1] = std::min(best_ms[rep & 1], trial(cand[rep & 1], false));
    const int block = best_ms[0] <= best_ms[1] ? cand[0] : cand[1];
    // k-space column blocks with that size: each member's own, or one width for all members (widths whose
    // LDS does not fit are skipped), each twice
    const int zcand[6] = {0, 8, 12, 16, 24, 32};
    float best_z_ms = std::min(best_ms[0], best_ms[1]);
    int best_z = keep_z;
    for (int rep = 0; rep < 2 && e == hipSuccess && rc == TILD_OK; ++rep)
        for (const int zc : zcand) {
            if (e != hipSuccess || rc != TILD_OK) break;
            if (zc != b->z_cols) {
                const hipError_t eb = build_batch_maps(b, zc);
                if (eb == hipErrorInvalidValue) continue;  // does not fit: skipped
                e = eb;
                if (e != hipSuccess) break;
            }
            const float ms = trial(block, false);
            if (ms < best_z_ms) {
                best_z_ms = ms;
                best_z = zc;
            }
        }
    if (e == hipSuccess && rc == TILD_OK && b->z_cols != best_z) e = build_batch_maps(b, best_z);
    float graph_ms = 1e30f;
    if (e == hipSuccess && rc == TILD_OK) (void)trial(block, true);
    for (int rep = 0; rep < 2 && e == hipSuccess && rc == TILD_OK; ++rep) graph_ms = std::min(graph_ms, trial(block, true));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    (void)hipFree(snap);
    if (rc != TILD_OK || e != hipSuccess) {
        b->B.plane_block = keep_block;
        b->use_graph = keep_graph;
        if (b->z_cols != keep_z) (void)build_batch_maps(b, keep_z);
        if (rc != TILD_OK) return b->fail(rc, "autotune: a trial step or the restore failed");
        return b->hip_fail(e, "autotune");
    }
    b->B.plane_block = block;
    b->use_graph = graph_ms <= best_z_ms;
    if (plane_block) *plane_block = b->B.plane_block;
    if (z_cols) *z_cols = b->z_cols;
    if (graph) *graph = b->use_graph ? 1 : 0;
    return TILD_OK;
}

TILD_API int tild_batch_set_graph(tild_batch* b, int32_t use_graph) {
    if (!b) return TILD_EINVAL;
    b->use_graph = use_graph != 0;
    return TILD_OK;
}

TILD_API int tild_batch_synchronize(tild_batch* b) {
    if (!b) return TILD_EINVAL;
    DeviceGuard g(b->device);
    const hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return b->hip_fail(e, "batch synchronize");
    for (tild_ctx* c : b->ctx) {
        const int rc = check_flag(c);
        if (rc != TILD_OK) return b->fail(rc, c->err);
    }
    return TILD_OK;
}

TILD_API const char* tild_batch_last_error(const tild_batch* b) {
    return b ? b->err.c_str() : g_create_error.c_str();
}

// ---------------------------------------------------------------- batches without allocations
//
// tild_batch_step_static steps a set of contexts as one batch with no batch
// object: the member descriptors, the unit maps and the bin-scan status words
// live in this file's `scratch` array, one copy per device, whose address is
// taken once per device with hipGetSymbolAddress.  The host side builds them
// in a fixed static staging buffer of the same size.  Nothing is allocated
// per call; concurrent calls on one device share the array and race.

static constexpr size_t kStaticScratchBytes = 1u << 20;  // 1 MiB per device
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

struct StaticSlot {
    void* ptr = nullptr;         // device address of `scratch` on this device
    hipEvent_t copied = nullptr;  // recorded after the staging buffer's upload
    bool copy_pending = false;
};
StaticSlot g_static[kMaxDevices];
std::mutex g_static_mu;
alignas(256) unsigned char g_static_stage[kStaticScratchBytes];  // host staging (guarded by g_static_mu)

__global__ void __launch_bounds__(256) k_zero_u64(unsigned long long* __restrict__ p, long long n) {
    const long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Per-device set-up on first use (the device is current): the scratch array's
// address and the event that guards the staging buffer.
hipError_t static_slot(int dev, StaticSlot** out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    StaticSlot& s = g_static[dev];
    if (!s.ptr) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        e = hipEventCreateWithFlags(&s.copied, hipEventDisableTiming);
        if (e != hipSuccess) return e;
        s.ptr = ptr;
    }
    *out = &s;
    return hipSuccess;
}

}  // namespace

TILD_API int tild_batch_step_static(tild_ctx* const* ctxs, int32_t n_ctx, int64_t n_steps, void* hip_stream) {
    auto bad = [&](int code, const std::string& why) {
        g_create_error = "batch_step_static: " + why;
        return code;
    };
    if (!ctxs || n_ctx < 1 || n_ctx > 65535) return bad(TILD_EINVAL, "needs 1..65535 contexts");
    if (n_steps < 0 || n_steps > 0x7fffffffLL) return bad(TILD_EINVAL, "n_steps must be in [0, 2^31)");
    const hipStream_t stream = (hipStream_t)hip_stream;
    const tild_ctx* c0 = ctxs[0];
    if (!c0) return bad(TILD_EINVAL, "NULL context");
    for (int32_t i = 0; i < n_ctx; ++i) {
        const tild_ctx* c = ctxs[i];
        if (!c) return bad(TILD_EINVAL, "NULL context");
        for (int32_t k = 0; k < i; ++k)
            if (ctxs[k] == c) return bad(TILD_EINVAL, "a context appears twice");
        if (c->device != c0->device) return bad(TILD_EINVAL, "contexts on different devices");
        if (c->L.stream != stream) return bad(TILD_EINVAL, "every member must use the stream passed in");
        if (c->L.precision != c0->L.precision || c->L.order != c0->L.order || c->p.flags != c0->p.flags ||
            c->L.ph.elec != c0->L.ph.elec)
            return bad(TILD_EINVAL, "contexts differ in precision, order, flags or the presence of charges");
        if (c->L.force_ad || c->L.ph.gjf) return bad(TILD_EINVAL, "batched steps use the ik route and Euler-Maruyama");
        if ((c->S.n + 255) / 256 > 65535) return bad(TILD_EINVAL, "a member has more than 16,776,960 beads");
        if (!c->have_pos) return bad(TILD_ESTATE, "a member's positions were never set");
    }
    if (n_steps == 0) return TILD_OK;
    // scratch layout: descriptors, unit maps (plane, c2r, zcol, bead, tile), scan status words + ticket
    size_t n_plane = 0, n_c2r = 0, n_zcol = 0, n_bead = 0, n_tile = 0;
    size_t lds_plane = 0, lds_z = 0;
    int max_plane = 0;
    for (int32_t r = 0; r < n_ctx; ++r) {
        const tild_ctx* c = ctxs[r];
        n_plane += 2 * (size_t)c->L.d.mz;
        n_c2r += 6 * (size_t)c->L.d.mz;
        n_zcol += (size_t)c->L.n_zblocks;
        n_bead += (size_t)((c->S.n + 255) / 256);
        n_tile += (size_t)((c->S.nbins + kScanBins - 1) / kScanBins);
        lds_plane = std::max(lds_plane, plane_lds_bytes(c->L));
        lds_z = std::max(lds_z, z_lds_bytes(c->L));
        max_plane = std::max(max_plane, c->L.d.mx * c->L.d.my);
    }
    const size_t nmap = n_plane + n_c2r + n_zcol + n_bead + n_tile;
    const size_t desc_bytes = ((size_t)n_ctx * sizeof(RepDesc) + 255) / 256 * 256;
    const size_t map_bytes = (nmap * sizeof(uint32_t) + 255) / 256 * 256;
    const size_t status_words = n_tile + 1;
    const size_t need = desc_bytes + map_bytes + status_words * sizeof(unsigned long long);
    if (need > kStaticScratchBytes)
        return bad(TILD_EINVAL, "the batch needs " + std::to_string(need) + " bytes of scratch; the limit is " +
                                    std::to_string(kStaticScratchBytes));
    std::lock_guard<std::mutex> lock(g_static_mu);
    DeviceGuard g(c0->device);
    StaticSlot* slot = nullptr;
    hipError_t e = static_slot(c0->device, &slot);
    if (e != hipSuccess) return bad(TILD_EHIP, std::string("scratch set-up: ") + hipGetErrorString(e));
    // the previous call's upload must have left the staging buffer
    if (slot->copy_pending) {
        e = hipEventSynchronize(slot->copied);
        if (e != hipSuccess) return bad(TILD_EHIP, std::string("staging wait: ") + hipGetErrorString(e));
        slot->copy_pending = false;
    }
    unsigned char* dev = static_cast<unsigned char*>(slot->ptr);
    RepDesc* h_desc = reinterpret_cast<RepDesc*>(g_static_stage);
    uint32_t* h_map = reinterpret_cast<uint32_t*>(g_static_stage + desc_bytes);
    unsigned long long* d_status = reinterpret_cast<unsigned long long*>(dev + desc_bytes + map_bytes);
    uint32_t* mp = h_map;
    uint32_t* mc = mp + n_plane;
    uint32_t* mz = mc + n_c2r;
    uint32_t* mb = mz + n_zcol;
    uint32_t* mt = mb + n_bead;
    size_t status_off = 0;
    for (int32_t r = 0; r < n_ctx; ++r) {
        const tild_ctx* c = ctxs[r];
        const Dims& d = c->L.d;
        const uint32_t hi = (uint32_t)r << 16;
        for (int u = 0; u < 2 * d.mz; ++u) *mp++ = hi | (uint32_t)u;
        for (int u = 0; u < 6 * d.mz; ++u) *mc++ = hi | (uint32_t)u;
        for (int u = 0; u < c->L.n_zblocks; ++u) *mz++ = hi | (uint32_t)u;
        for (long long u = 0; u < (c->S.n + 255) / 256; ++u) *mb++ = hi | (uint32_t)u;
        const int ntiles = (c->S.nbins + kScanBins - 1) / kScanBins;
        for (int u = 0; u < ntiles; ++u) *mt++ = hi | (uint32_t)u;
        RepDesc& R = h_desc[r];
        std::memset(&R, 0, sizeof(R));
        R.d = c->L.d;
        R.px = c->L.px;
        R.py = c->L.py;
        R.pz = c->L.pz;
        R.ph = c->L.ph;
        R.S = c->S;
        R.S.scan_status = d_status + status_off;
        R.z_cols = c->L.z_cols;
        R.n_zblocks = c->L.n_zblocks;
        R.ntiles = ntiles;
        R.step0 = (uint64_t)c->step;
        status_off += (size_t)ntiles;
    }
    Launch L = c0->L;
    L.stream = stream;
    BatchMaps B{};
    B.reps = reinterpret_cast<const RepDesc*>(dev);
    B.plane = reinterpret_cast<const uint32_t*>(dev + desc_bytes);
    B.c2r = B.plane + n_plane;
    B.zcol = B.c2r + n_c2r;
    B.bead = B.zcol + n_zcol;
    B.tile = B.bead + n_bead;
    B.n_plane = (int)n_plane;
    B.n_c2r = (int)n_c2r;
    B.n_zcol = (int)n_zcol;
    B.n_bead = (int)n_bead;
    B.n_tile = (int)n_tile;
    B.ticket = d_status + n_tile;
    B.plane_block = max_plane <= 96 * 96 ? 256 : 512;
    e = hipMemcpyAsync(dev, g_static_stage, desc_bytes + nmap * sizeof(uint32_t), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipEventRecord(slot->copied, stream);
    if (e == hipSuccess) slot->copy_pending = true;
    // the scan's status words and ticket start at zero: the previous call left later epochs in them
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)((status_words + 255) / 256)), dim3(256), 0, stream, d_status,
                           (long long)status_words);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = configure_batch_attributes(L, lds_plane, lds_z);
    if (e == hipSuccess) e = launch_batch_noise(L, B);
    for (int64_t s = 0; e == hipSuccess && s < n_steps; ++s) e = launch_batch_step(L, B, (int)s, lds_plane, lds_z);
    if (e != hipSuccess) {
        for (int32_t r = 0; r < n_ctx; ++r) ctxs[r]->noise_ready = -1;
        return bad(TILD_EHIP, std::string("batch step: ") + hipGetErrorString(e));
    }
    for (int32_t r = 0; r < n_ctx; ++r) {
        tild_ctx* c = ctxs[r];
        if (n_steps & 1) {
            std::swap(c->S.qshift, c->S.qshift_next);
            std::swap(c->S.nbr, c->S.nbr_old);
        }
        c->step += n_steps;
        c->noise_ready = c->step;
    }
    return TILD_OK;
}

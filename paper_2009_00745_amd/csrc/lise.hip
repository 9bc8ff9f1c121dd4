// Host side of the MI355X TDSLDA step library: context, device buffers, FFT
// plans, the series-expansion start-up and the two-phase ABM schedule, and
// the C-ABI declared in include/lise.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "lise.h"
#include "lise_device.hpp"
#define LISE_PLAN_HAVE_DEVICE_TYPES 1
#include "lise_plan.hpp"
#include "lise_fast.hpp"
#include "lise_mfma.hpp"
#include "lise_cube.hpp"
#include <type_traits>

using namespace lise;
using lise::plan::factorize;
using lise::plan::make_plan;
using lise::plan::mfma_side;
using lise::plan::kinetic_matrix_bf16;

namespace {

constexpr int kThreads = 256;
const char* kVersion = "lise-mi355x 0.1 (gfx950)";
constexpr int kBatchPeriod = 4;   // ABM steps after which the buffer ring repeats
constexpr int kPlaneJg = 32;      // default qpwfs per workgroup row of the plane kernels
constexpr int kCubeJg = 16;       // ... of the single-pass kernel (one workgroup holds a whole qpwf)
constexpr int kZdJg = 128;        // ... of the plane kernel with the z-term inside (measured 64-256 alike)
constexpr size_t kDescRowsOffset = 1024;   // the one-entry table of a single system: descriptor, then rows

// Staging memory of lise_apply_h_noalloc: one fixed array per GPU, held until
// the process ends, shared by every context on that GPU.  Host code never
// uses the name `scratch` as an address (in host code it is a stand-in, not
// device memory); it uses the address hipGetSymbolAddress returned for the
// device, recorded once per device by lise_init.
constexpr size_t kScratchBytes = (size_t)LISE_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
void* g_scratch_addr[kMaxDevices] = {};
std::mutex g_scratch_mu;

struct Prof {
    bool on = false;
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Rec { int cls; hipEvent_t a, b; };
    std::vector<Rec> recs;
    double total_ms[5] = {0, 0, 0, 0, 0};
    long long count[5] = {0, 0, 0, 0, 0};
    bool overflow = false;
};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct lise_ctx {
    lise_lattice lat;
    lise_functional fn;
    long long M = 0, N = 0;
    int C = 2;
    int prec = LISE_FP64;
    size_t esz = 16;          // bytes per complex element of the state
    long long per = 0;        // elements per qpwf = C * N
    hipStream_t stream = nullptr;
    int device = 0;
    size_t lds_limit = 65536;

    void* buf[7] = {nullptr};  // 0,1: y ring; 2..5: derivative ring; 6: p - c
    void* G = nullptr;         // z-axis scratch, chunk qpwfs (current buffer)
    void* Gbuf[2] = {nullptr, nullptr};   // double buffer when the z kernel runs ahead
    long long g_cap = 0;       // qpwfs each G buffer holds
    hipStream_t s2 = nullptr;  // internal stream of the z-axis kernel (default priority)
    hipStream_t cap = nullptr; // internal stream graphs are captured on (never the null stream)
    hipEvent_t ev_cap = nullptr;
    hipEvent_t ev_start = nullptr, ev_kz[2] = {nullptr, nullptr}, ev_kp[2] = {nullptr, nullptr};
    int overlap = 1;
    int mfma_mode = 0;         // precision LISE_FP32_MFMA
    double* dpart = nullptr;   // density partial slots
    int slot_cap = 0;
    double* dens_cur = nullptr;
    double* dens_tmp = nullptr;
    double* V_cur = nullptr;
    double* D_cur = nullptr;
    double* V_tmp = nullptr;
    double* D_tmp = nullptr;
    void* tw = nullptr;
    void* ah_buf = nullptr;    // staging of lise_apply_h (one piece, kept)
    size_t ah_cap = 0;
    void* scratch_dev = nullptr;  // this device's address of `scratch` (lise_apply_h_noalloc)
    void* cube_desc = nullptr;    // one-entry descriptor table of the single-pass kernel
    void* tzm = nullptr;          // dense z-term operator T_z (nz x nz, the state's type)
    double* red = nullptr;     // reduction partials (observables)
    long long red_cap = 0;
    double* pz_part = nullptr;  // per-workgroup z-momentum sums (observables)
    long long pz_cap = 0;
    double* norms = nullptr;
    double* norms0 = nullptr;
    int* bad = nullptr;
    double* dtime = nullptr;   // device copy of t (advanced by tick_kernel)
    AxisPlan px, py, pz;

    // tuning
    int chunk = 0, jg = 32, fused_mode = 0, generic = 0;   // fused_mode: -1 never, 0 auto, 1 prefer
    int jg_user = 0;            // jgroup the caller set (0: the path's default)
    int single_pass = 0;        // -1 never, 0 auto, 1 prefer the single-pass ABM kernel
    int z_dense_user = 0;       // -1 never, 0 default, 1 the in-kernel z-term where available
    bool zdense = false;        // ABM phases: plane kernel with the z-term in the kernel
    int zl_user = 0;            // lanes per z-column the caller set (0: default)
    int zl = 1;                 // lanes per z-column of the register-FFT z kernel (1, 2 or 4)
    bool cube = false;          // ABM phases by the single-pass kernel (lise_cube.hpp)
    bool stream_hint = false;   // z kernel takes nontemporal hints (as the plane kernel does)
    bool fused = false;
    int zb = 1, yb = 1, ppt = 4;
    bool fast_xy = false, fast_z = false;   // size-specialised register-FFT kernels
    bool mfma_xy = false;                   // split-bf16 MFMA plane kernel (LISE_FP32_MFMA)
    short* dkin = nullptr;                  // bf16 hi/lo of the 1D kinetic matrix
    int tw_full_xy = -1, tw_full_z = -1;    // offsets of W_n^j tables (j < n)

    // state
    std::vector<unsigned char> set_mask;   // per qpwf: written since the last reset
    long long n_set = 0;                   // qpwfs marked in set_mask
    bool dens_valid = false;
    double g_used = 0.0;       // coupling of Delta = -g kappa (bare or regularised)
    int remove_phase = 0;      // Eq. (sp_en): evolve with H - eta_j
    double* eta = nullptr;     // [M] eta_j of the vector the current H application acts on
    double* eta_part = nullptr;  // partial sums of the eta pass: [chunk][plane blocks] ([..][waves] forward-only)
    long long eta_part_cap = 0;
    double* ez_part[2] = {nullptr, nullptr};  // z-kinetic partials of the eta pass, per G buffer
    long long ez_cap = 0;
    bool hist = false;
    bool norms0_valid = false;
    double dt_hist = 0.0;
    double t = 0.0;
    long long step = 0;
    int iy = 0;   // buf index of y_n (0 or 1)
    int dn = 0;   // derivative slot receiving y'_n (0..3)

    Prof prof;
    bool capturing = false;
    int use_graph = 0;            // lise_step replays a captured 4-step graph
    hipGraphExec_t gexec = nullptr;
    long long gsig = -1;          // ring state the graph was captured in
    long long config_version = 0;
    char err[512] = {0};
};

namespace {

int fail(lise_ctx* c, int code, const char* fmt, ...) {
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(c->err, sizeof(c->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

#define HIPCHK(ctx, call)                                                                       \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess) return fail(ctx, LISE_E_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define CHK(call)                  \
    do {                           \
        int rc_ = (call);          \
        if (rc_ != LISE_OK) return rc_; \
    } while (0)

template <typename T>
cpx<T>* S(lise_ctx* c, int i) { return reinterpret_cast<cpx<T>*>(c->buf[i]); }

// ---- profiling -------------------------------------------------------------
void prof_begin(lise_ctx* c, int cls, hipEvent_t* ev, hipStream_t st) {
    *ev = nullptr;
    if (!c->prof.on || c->capturing) return;
    if (c->prof.used + 2 > c->prof.pool.size()) {
        c->prof.overflow = true;
        return;
    }
    *ev = c->prof.pool[c->prof.used];
    (void)hipEventRecord(*ev, st);
    (void)cls;
}
void prof_begin(lise_ctx* c, int cls, hipEvent_t* ev) { prof_begin(c, cls, ev, c->stream); }
void prof_end(lise_ctx* c, int cls, hipEvent_t a, hipStream_t st) {
    if (!a) return;
    hipEvent_t b = c->prof.pool[c->prof.used + 1];
    c->prof.used += 2;
    (void)hipEventRecord(b, st);
    c->prof.recs.push_back({cls, a, b});
}
void prof_end(lise_ctx* c, int cls, hipEvent_t a) { prof_end(c, cls, a, c->stream); }

int check_launch(lise_ctx* c, const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, LISE_E_HIP, "launch of %s failed: %s", what, hipGetErrorString(e));
    return LISE_OK;
}

// ---- allocation -------------------------------------------------------------
int dalloc(lise_ctx* c, void** p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(c, LISE_E_NOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    }
    return LISE_OK;
}

void dfree(void** p) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
}

size_t kp_lds_bytes(const lise_ctx* c, int zb) { return 2ull * 2ull * (size_t)zb * c->lat.nx * c->lat.ny * c->esz; }
size_t kz_lds_bytes(const lise_ctx* c, int yb) { return 2ull * (size_t)c->lat.nz * yb * c->lat.nx * c->esz; }

bool fast_side(int n) {
    return n == 8 || n == 16 || n == 20 || n == 24 || n == 32 || n == 48 || n == 64;
}

size_t fast_kp_lds(const lise_ctx* c) {
    const size_t n = c->lat.nx;
    const bool natural = plane_natural_of((int)c->esz / 2, (int)n);
    return (n + 2 * n * (n + 1) + (natural ? 2 * n * n : 0)) * c->esz;
}

// workgroups along z of one plane-kernel launch (= partial sums per qpwf of
// the reducing modes)
int plane_grid_x(const lise_ctx* c) {
    if (c->fast_xy || c->mfma_xy) return c->lat.nz;
    return c->lat.nz / c->zb;
}

// The forward-only pass walks kEtaJg qpwfs per workgroup and writes one
// partial sum per wave, plane block and qpwf.
constexpr int kEtaJg = 4;
long long etaxy_parts(const lise_ctx* c) {
    return (long long)plane_grid_x(c) * (plane_block_of((int)c->esz / 2, c->lat.nx) / 64);
}

// Allow every kernel that takes dynamic LDS to use the device's whole LDS,
// once per process (outside any stream capture).
template <typename T, int NS>
void set_fast_attrs(int lim) {
    (void)hipFuncSetAttribute((const void*)kp_fast<T, NS, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)kp_fast<T, NS, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)kp_fast<T, NS, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)kp_fast<T, NS, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)kp_fast<T, NS, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)kp_fast<T, NS, 5>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)kp_fast_batch<T, NS, KP_ABM1>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)kp_fast_batch<T, NS, KP_ABM2>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    if constexpr (zd_side((int)sizeof(T), NS)) {
        (void)hipFuncSetAttribute((const void*)kp_fast_zd<T, NS, KP_ABM1>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        (void)hipFuncSetAttribute((const void*)kp_fast_zd<T, NS, KP_ABM2>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    }
    if constexpr (cube_side((int)sizeof(T), NS)) {
        (void)hipFuncSetAttribute((const void*)kc_fast_batch<T, NS, KP_ABM1>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        (void)hipFuncSetAttribute((const void*)kc_fast_batch<T, NS, KP_ABM2>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    }
}

template <typename T>
void set_type_attrs(int lim) {
    set_fast_attrs<T, 8>(lim);
    set_fast_attrs<T, 16>(lim);
    set_fast_attrs<T, 20>(lim);
    set_fast_attrs<T, 24>(lim);
    set_fast_attrs<T, 32>(lim);
    set_fast_attrs<T, 48>(lim);
    set_fast_attrs<T, 64>(lim);
    const void* g[] = {(const void*)kp_kernel<T, 0, 4>, (const void*)kp_kernel<T, 1, 4>, (const void*)kp_kernel<T, 2, 4>,
                       (const void*)kp_kernel<T, 3, 4>, (const void*)kp_kernel<T, 0, 16>, (const void*)kp_kernel<T, 1, 16>,
                       (const void*)kp_kernel<T, 2, 16>, (const void*)kp_kernel<T, 3, 16>, (const void*)kp_kernel<T, 4, 4>,
                       (const void*)kp_kernel<T, 4, 16>, (const void*)kz_kernel<T>,
                       (const void*)current_xy_kernel<T, 4>, (const void*)current_xy_kernel<T, 16>,
                       (const void*)current_z_kernel<T, 4>, (const void*)current_z_kernel<T, 16>};
    for (const void* f : g) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
}

template <int NS>
void set_mfma_attrs(int lim) {
    (void)hipFuncSetAttribute((const void*)kp_mfma<NS, 0>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)kp_mfma<NS, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)kp_mfma<NS, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)kp_mfma<NS, 3>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
    (void)hipFuncSetAttribute((const void*)kp_mfma<NS, 4>, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
}

void set_all_attrs(int lim) {
    static bool done = false;
    if (done) return;
    done = true;
    set_type_attrs<double>(lim);
    set_type_attrs<float>(lim);
    set_mfma_attrs<16>(lim);
    set_mfma_attrs<32>(lim);
    set_mfma_attrs<48>(lim);
    set_mfma_attrs<64>(lim);
}

// Whether the single-pass ABM kernel covers the lattice (after the
// register-FFT flags are set).
bool cube_eligible(const lise_ctx* c) {
    const int n = c->lat.nx;
    return c->fast_xy && c->fast_z && n == c->lat.ny && n == c->lat.nz && cube_side((int)c->esz / 2, n) &&
           cube_lds_of((int)c->esz / 2, n) <= c->lds_limit && !c->remove_phase;
}

// The plane kernel with the z-term in the kernel (kp_fast_zd): cubic lattices
// on the register-FFT kernels, the ABM phases without phase removal.
bool zdense_eligible(const lise_ctx* c) {
    const int n = c->lat.nx;
    const int esz = (int)c->esz / 2;
    const size_t lds = (size_t)(n + 2 * n * (n + 1)) * c->esz + (size_t)kZdPlanes * n * esz +
                       (size_t)kZdPlanes * 3 * n * n * sizeof(double);
    return c->fast_xy && c->fast_z && n == c->lat.ny && n == c->lat.nz && !c->remove_phase &&
           (n == 16 || n == 32) && zd_side(esz, n) && lds <= c->lds_limit;
}

// T_z of Eq. (tdslda)'s kinetic term along z on the lattice: the z-axis
// kernel multiplies the spectrum by c_z m^2 (m the signed index, Nyquist
// kept) between a forward and an inverse transform of nz points, so
// T_z[z][z'] = c_z sum_k m_k^2 cos(2 pi k (z - z') / nz) with
// c_z = (2 pi^2 / L_z^2) / nz (the sine parts cancel: m_k^2 is even in k).
// Summed in long double and rounded once to the state's type.
template <typename T>
int build_tzm(lise_ctx* c) {
    const int nz = c->lat.nz;
    const long double pi = 3.141592653589793238462643383279502884L;
    const long double lz = (long double)nz * c->lat.a;
    const long double cz = 2.0L * pi * pi / (lz * lz) / nz;
    std::vector<long double> row(nz);
    for (int d = 0; d < nz; ++d) {
        long double sum = 0.0L;
        for (int k = 0; k < nz; ++k) {
            const long double m = (2 * k < nz) ? k : k - nz;
            sum += m * m * cosl(2.0L * pi * (long double)((long long)k * d % nz) / nz);
        }
        row[d] = cz * sum;
    }
    std::vector<T> h((size_t)nz * nz);
    for (int z = 0; z < nz; ++z)
        for (int zp = 0; zp < nz; ++zp) h[(size_t)z * nz + zp] = T(row[(z - zp + nz) % nz]);
    CHK(dalloc(c, &c->tzm, h.size() * sizeof(T)));
    HIPCHK(c, hipMemcpy(c->tzm, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return LISE_OK;
}

// Choose launch geometry and (re)allocate scratch for the current tuning.
int configure(lise_ctx* c) {
    c->config_version += 1;
    const int nx = c->lat.nx, ny = c->lat.ny, nz = c->lat.nz;
    const long long nxy = (long long)nx * ny;
    // fused: the whole cube of one component pair in LDS (two buffers)
    c->fused = false;
    // auto: the whole-cube LDS kernel only where the register-FFT kernels do
    // not cover the lattice (they measured faster where both exist)
    const bool reg_fft = !c->generic && nx == ny && fast_side(nx) && fast_side(nz) && fast_kp_lds(c) <= c->lds_limit &&
                         c->tw_full_xy >= 0 && c->tw_full_z >= 0;
    const bool want_fused = c->fused_mode > 0 || (c->fused_mode == 0 && !reg_fft);
    if (want_fused && !c->mfma_mode && kp_lds_bytes(c, nz) <= c->lds_limit && c->N <= 16LL * kThreads)
        c->fused = true;
    if (c->fused) {
        c->zb = nz;
    } else {
        int zb = 1;
        for (int d = 1; d <= nz; ++d)
            if (nz % d == 0 && d * nxy >= kThreads && kp_lds_bytes(c, d) <= c->lds_limit) { zb = d; break; }
        c->zb = zb;
        int yb = 1;
        for (int d = ny; d >= 1; --d)
            if (ny % d == 0 && (long long)d * nx * nz <= (c->prec == LISE_FP64 ? 2048 : 4096) &&
                kz_lds_bytes(c, d) <= c->lds_limit) { yb = d; break; }
        c->yb = yb;
    }
    c->mfma_xy = c->mfma_mode && !c->fused && nx == ny && mfma_side(nx) && c->dkin;
    c->fast_xy = !c->mfma_xy && !c->fused && !c->generic && nx == ny && fast_side(nx) &&
                 fast_kp_lds(c) <= c->lds_limit && c->tw_full_xy >= 0;
    c->fast_z = !c->fused && !c->generic && fast_side(nz) && c->tw_full_z >= 0;
    if (c->fast_xy || c->mfma_xy) c->zb = 1;
    c->zl = (c->zl_user > 0 && kz_lanes_valid(nz, c->zl_user)) ? c->zl_user : kz_lanes_of(nz);
    // single-pass ABM kernel: the whole pair of component cubes in LDS; by
    // default where it measured faster than the two kernels
    c->cube = cube_eligible(c) &&
              (c->single_pass > 0 || (c->single_pass == 0 && cube_auto_of((int)c->esz / 2, nx)));
    // in-kernel z-term: by default where it measured faster than the two
    // kernels (float64 side 32: 28.3 against 30.5 ms per step at 8192 qpwfs;
    // float32 side 32 slower, 19.0 against 16.5)
    c->zdense = !c->cube && zdense_eligible(c) &&
                (c->z_dense_user > 0 || (c->z_dense_user == 0 && c->prec == LISE_FP64 && nx == 32));
    c->jg = c->jg_user > 0 ? c->jg_user : (c->cube ? kCubeJg : (c->zdense ? kZdJg : kPlaneJg));
    if (c->zdense && !c->tzm) CHK(c->prec == LISE_FP64 ? build_tzm<double>(c) : build_tzm<float>(c));
    static_assert(sizeof(KPArgs<double>) <= kDescRowsOffset, "descriptor table layout");
    if (c->cube && !c->cube_desc) CHK(dalloc(c, &c->cube_desc, kDescRowsOffset + 64));
    c->stream_hint = c->mfma_xy || (c->fast_xy && plane_stream_hint_of(c->esz / 2, nx));
    // the generic LDS kernels must fit where they are the ones that run
    if (!c->fused && !c->fast_xy && !c->mfma_xy && kp_lds_bytes(c, c->zb) > c->lds_limit)
        return fail(c, LISE_E_UNSUPPORTED, "xy-plane %dx%d does not fit in LDS (%zu > %zu bytes)", nx, ny,
                    kp_lds_bytes(c, c->zb), c->lds_limit);
    if (!c->fused && !c->fast_z && kz_lds_bytes(c, c->yb) > c->lds_limit)
        return fail(c, LISE_E_UNSUPPORTED, "xz-tile %dx%d does not fit in LDS", nz, nx);
    const long long P = (long long)c->zb * nxy;
    const long long ppt = (P + kThreads - 1) / kThreads;
    if (ppt > 16) return fail(c, LISE_E_UNSUPPORTED, "plane stack of %lld points exceeds 16 per thread", P);
    c->ppt = ppt <= 4 ? 4 : 16;

    long long chunk = c->chunk > 0 ? c->chunk : 0;
    if (chunk <= 0) {
        // default: a z-scratch of ~4 GiB (two with the z kernel overlapped).
        // Larger launches measured faster than cache-sized ones, and enough
        // plane workgroups per launch keep its tail short: 48^3 float32 took
        // 119 ms per step at 606 qpwfs per launch (1 GiB), 109 at 2048-16384
        const long long per_bytes = c->per * (long long)c->esz;
        chunk = std::max<long long>(c->jg, (4LL << 30) / std::max<long long>(per_bytes, 1));
    }
    chunk = std::min<long long>(chunk, c->M);
    chunk = std::max<long long>(chunk, 1);
    c->chunk = (int)chunk;
    const int slots = (int)((chunk + c->jg - 1) / c->jg);
    const long long dens_slots = std::max<long long>(slots, (c->M + c->jg - 1) / c->jg);
    if (!c->fused && c->g_cap < chunk) {
        dfree(&c->Gbuf[0]);
        dfree(&c->Gbuf[1]);
        c->G = nullptr;
        c->g_cap = 0;
        CHK(dalloc(c, &c->Gbuf[0], (size_t)chunk * c->per * c->esz));
        if (c->overlap) CHK(dalloc(c, &c->Gbuf[1], (size_t)chunk * c->per * c->esz));
        c->g_cap = chunk;
    }
    if (!c->fused && c->overlap && !c->Gbuf[1]) CHK(dalloc(c, &c->Gbuf[1], (size_t)c->g_cap * c->per * c->esz));
    c->G = c->Gbuf[0];
    if (c->slot_cap < dens_slots) {
        dfree(reinterpret_cast<void**>(&c->dpart));
        CHK(dalloc(c, reinterpret_cast<void**>(&c->dpart), (size_t)dens_slots * 3 * c->N * sizeof(double)));
        c->slot_cap = (int)dens_slots;
    }
    if (c->remove_phase) {
        const long long need =
            c->chunk * std::max<long long>(nz / c->zb, c->fast_xy && c->fast_z ? etaxy_parts(c) : 0);
        if (c->eta_part_cap < need) {
            dfree(reinterpret_cast<void**>(&c->eta_part));
            CHK(dalloc(c, reinterpret_cast<void**>(&c->eta_part), (size_t)need * sizeof(double)));
            c->eta_part_cap = need;
        }
        if (!c->eta) CHK(dalloc(c, reinterpret_cast<void**>(&c->eta), (size_t)c->M * sizeof(double)));
        if (c->fast_xy && c->fast_z) {
            const long long nez = c->chunk * (long long)c->C * nxy * c->zl;
            if (c->ez_cap < nez) {
                for (int b = 0; b < 2; ++b) {
                    dfree(reinterpret_cast<void**>(&c->ez_part[b]));
                    CHK(dalloc(c, reinterpret_cast<void**>(&c->ez_part[b]), (size_t)nez * sizeof(double)));
                }
                c->ez_cap = nez;
            }
        }
    }
    return LISE_OK;
}

FieldParams field_params(const lise_ctx* c) {
    FieldParams f;
    f.nx = c->lat.nx;
    f.ny = c->lat.ny;
    f.nz = c->lat.nz;
    f.a = c->lat.a;
    f.beta = c->fn.beta;
    f.g = c->g_used;
    f.frozen = c->fn.frozen;
    f.U0 = c->fn.U0;
    f.D0re = c->fn.Delta0_re;
    f.D0im = c->fn.Delta0_im;
    f.extA = c->fn.ext_A;
    f.extw = c->fn.ext_w;
    f.r0x = c->fn.ext_r0[0];
    f.r0y = c->fn.ext_r0[1];
    f.r0z = c->fn.ext_r0[2];
    f.t_on = c->fn.ext_t_on;
    return f;
}

// ---- kernel launchers ---------------------------------------------------------

template <typename T>
KPArgs<T> kp_base(lise_ctx* c) {
    KPArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.nx = c->lat.nx;
    a.ny = c->lat.ny;
    a.nz = c->lat.nz;
    a.C = c->C;
    a.npair = c->C / 2;
    a.zb = c->zb;
    a.jg = c->jg;
    a.fused = c->fused ? 1 : 0;
    a.px = c->px;
    a.py = c->py;
    a.pz = c->pz;
    a.tw = reinterpret_cast<const cpx<T>*>(c->tw);
    const double pi = 3.14159265358979323846;
    const double tsize = c->fused ? (double)c->N : (double)c->lat.nx * c->lat.ny;
    const double lx = c->lat.nx * c->lat.a, ly = c->lat.ny * c->lat.a, lz = c->lat.nz * c->lat.a;
    a.cx = T(2.0 * pi * pi / (lx * lx) / tsize);
    a.cy = T(2.0 * pi * pi / (ly * ly) / tsize);
    a.cz = T(2.0 * pi * pi / (lz * lz) / tsize);
    if (c->C == 2) {
        a.ca[0] = 0; a.cb[0] = 1; a.sgn[0] = 1;
        a.mu_a[0] = a.mu_b[0] = c->fn.mu_up;
        a.w = c->fn.w;
    } else {
        a.ca[0] = 0; a.cb[0] = 3; a.sgn[0] = 1; a.mu_a[0] = c->fn.mu_up; a.mu_b[0] = c->fn.mu_dn;
        a.ca[1] = 1; a.cb[1] = 2; a.sgn[1] = -1; a.mu_a[1] = c->fn.mu_dn; a.mu_b[1] = c->fn.mu_up;
        a.w = 1.0;
    }
    a.dpart = c->dpart;
    return a;
}

template <typename T, int MODE, int NS>
void launch_kp_fast_n(lise_ctx* c, const KPArgs<T>& a, dim3 grid) {
    constexpr int block = plane_block<T, NS>();
    const size_t lds = std::max(kp_fast_lds<T, NS>(), (size_t)block * sizeof(double));
    hipLaunchKernelGGL((kp_fast<T, NS, MODE>), grid, dim3(block), lds, c->stream, a,
                       reinterpret_cast<const cpx<T>*>(c->tw) + c->tw_full_xy);
}

template <typename T, int MODE, int NS>
void launch_kp_zd_n(lise_ctx* c, const KPArgs<T>& a, int rows) {
    if constexpr (zd_side((int)sizeof(T), NS)) {
        constexpr int block = plane_block<T, NS>();
        constexpr size_t lds = kpzd_lds<T, NS>();
        hipLaunchKernelGGL((kp_fast_zd<T, NS, MODE>), dim3((unsigned)(NS / kZdPlanes * rows)), dim3(block), lds,
                           c->stream, a, reinterpret_cast<const cpx<T>*>(c->tw) + c->tw_full_xy, rows);
    }
}

// The ABM phases on the plane kernel with the z-term in the kernel: no
// z-axis launch, no z-term scratch.
template <typename T, int MODE>
int launch_kpzd_t(lise_ctx* c, KPArgs<T> a, long long j0, int k, int cls) {
    a.j0 = j0;
    a.kcount = k;
    a.G = nullptr;
    a.tzm = reinterpret_cast<const T*>(c->tzm);
    if (!a.tzm) return fail(c, LISE_E_STATE, "z-term operator table is not allocated");
    const int rows = (k + a.jg - 1) / a.jg;
    hipEvent_t ev;
    prof_begin(c, cls, &ev);
    switch (c->lat.nx) {
        case 16: launch_kp_zd_n<T, MODE, 16>(c, a, rows); break;
        default: launch_kp_zd_n<T, MODE, 32>(c, a, rows); break;
    }
    prof_end(c, cls, ev);
    return check_launch(c, "kp_fast_zd");
}

template <int MODE, int NS>
void launch_kp_mfma_n(lise_ctx* c, const KPArgs<float>& a, dim3 grid) {
    constexpr int block = mfma_block<NS>();
    const size_t lds = std::max(kp_mfma_lds<NS>(), (size_t)block * sizeof(double));
    hipLaunchKernelGGL((kp_mfma<NS, MODE>), grid, dim3(block), lds, c->stream, a, c->dkin);
}

template <typename T, int MODE>
int launch_kp_t(lise_ctx* c, KPArgs<T>& a, long long j0, int k, int cls) {
    a.j0 = j0;
    a.kcount = k;
    if constexpr (MODE == KP_ETAXY) {
        // the forward-only eta pass exists for the register-FFT plane kernel only
        if (!c->fast_xy) return fail(c, LISE_E_STATE, "forward-only eta pass without the register-FFT plane kernel");
    }
    if constexpr (std::is_same<T, float>::value && MODE != KP_ETAXY) {
        if (c->mfma_xy) {
            dim3 grid(c->lat.nz, (k + a.jg - 1) / a.jg);
            hipEvent_t ev;
            prof_begin(c, cls, &ev);
            switch (c->lat.nx) {
                case 16: launch_kp_mfma_n<MODE, 16>(c, a, grid); break;
                case 32: launch_kp_mfma_n<MODE, 32>(c, a, grid); break;
                case 48: launch_kp_mfma_n<MODE, 48>(c, a, grid); break;
                default: launch_kp_mfma_n<MODE, 64>(c, a, grid); break;
            }
            prof_end(c, cls, ev);
            return check_launch(c, "kp_mfma");
        }
    }
    if (c->fast_xy) {
        dim3 grid((unsigned)plane_grid_x(c), (k + a.jg - 1) / a.jg);
        hipEvent_t ev;
        prof_begin(c, cls, &ev);
        switch (c->lat.nx) {
            case 8: launch_kp_fast_n<T, MODE, 8>(c, a, grid); break;
            case 16: launch_kp_fast_n<T, MODE, 16>(c, a, grid); break;
            case 20: launch_kp_fast_n<T, MODE, 20>(c, a, grid); break;
            case 24: launch_kp_fast_n<T, MODE, 24>(c, a, grid); break;
            case 32: launch_kp_fast_n<T, MODE, 32>(c, a, grid); break;
            case 48: launch_kp_fast_n<T, MODE, 48>(c, a, grid); break;
            default: launch_kp_fast_n<T, MODE, 64>(c, a, grid); break;
        }
        prof_end(c, cls, ev);
        return check_launch(c, "kp_fast");
    }
    if constexpr (MODE == KP_ETAXY) {
        return LISE_E_STATE;   // not reached (checked above)
    } else {
        dim3 grid(c->lat.nz / c->zb, (k + a.jg - 1) / a.jg);
        // the kinetic-energy mode reuses LDS for a 256-double reduction
        const size_t lds = std::max(kp_lds_bytes(c, c->zb), (size_t)kThreads * sizeof(double));
        hipEvent_t ev;
        prof_begin(c, cls, &ev);
        if (c->ppt == 4) {
            hipLaunchKernelGGL((kp_kernel<T, MODE, 4>), grid, dim3(kThreads), lds, c->stream, a);
        } else {
            hipLaunchKernelGGL((kp_kernel<T, MODE, 16>), grid, dim3(kThreads), lds, c->stream, a);
        }
        prof_end(c, cls, ev);
        return check_launch(c, "kp_kernel");
    }
}

// nt: nontemporal hints on the column loads and scratch stores, taken where
// the plane kernel of the lattice takes them (whole-line plane rows; small
// lattices keep the default cache policy throughout)
template <typename T, int NZ, bool NT, int L>
void launch_kz_fast_l(const KZFastArgs<T>& f, hipStream_t st) {
    if constexpr (kz_lanes_valid(NZ, L)) {
        const long long threads = f.ncols * L;
        dim3 grid((unsigned)((threads + kThreads - 1) / kThreads));
        if constexpr (L > 1)
            hipLaunchKernelGGL((kz_lanes_kernel<T, NZ, L, NT>), grid, dim3(kThreads), 0, st, f);
        else
            hipLaunchKernelGGL((kz_fast<T, NZ, NT>), grid, dim3(kThreads), 0, st, f);
    }
}

// zl: lanes per column (1, 2 or 4; configure keeps only valid values)
template <typename T, int NZ, bool NT>
void launch_kz_fast_nt(const KZFastArgs<T>& f, hipStream_t st, int zl) {
    if (zl == 4) launch_kz_fast_l<T, NZ, NT, 4>(f, st);
    else if (zl == 2) launch_kz_fast_l<T, NZ, NT, 2>(f, st);
    else launch_kz_fast_l<T, NZ, NT, 1>(f, st);
}

template <typename T, int NZ>
void launch_kz_fast_n(const KZFastArgs<T>& f, hipStream_t st, bool nt, int zl) {
    if (nt)
        launch_kz_fast_nt<T, NZ, true>(f, st, zl);
    else
        launch_kz_fast_nt<T, NZ, false>(f, st, zl);
}

template <typename T>
int launch_kz_t(lise_ctx* c, const cpx<T>* in, long long j0, int k, void* Gdst, hipStream_t st,
                double* ezpart = nullptr) {
    if (c->fast_z) {
        KZFastArgs<T> f;
        f.nxy = (long long)c->lat.nx * c->lat.ny;
        f.ncols = (long long)k * c->C * f.nxy;
        f.j0 = j0;
        f.C = c->C;
        const double pi = 3.14159265358979323846;
        const double lz = c->lat.nz * c->lat.a;
        f.cz = T(2.0 * pi * pi / (lz * lz) / c->lat.nz);
        f.tw = reinterpret_cast<const cpx<T>*>(c->tw) + c->tw_full_z;
        f.in = in;
        f.G = reinterpret_cast<cpx<T>*>(Gdst);
        f.ezpart = ezpart;
        f.nu = c->C == 2 ? 1 : 2;
        hipEvent_t ev;
        prof_begin(c, 1, &ev, st);
        switch (c->lat.nz) {
            case 8: launch_kz_fast_n<T, 8>(f, st, c->stream_hint, c->zl); break;
            case 16: launch_kz_fast_n<T, 16>(f, st, c->stream_hint, c->zl); break;
            case 20: launch_kz_fast_n<T, 20>(f, st, c->stream_hint, c->zl); break;
            case 24: launch_kz_fast_n<T, 24>(f, st, c->stream_hint, c->zl); break;
            case 32: launch_kz_fast_n<T, 32>(f, st, c->stream_hint, c->zl); break;
            case 48: launch_kz_fast_n<T, 48>(f, st, c->stream_hint, c->zl); break;
            default: launch_kz_fast_n<T, 64>(f, st, c->stream_hint, c->zl); break;
        }
        prof_end(c, 1, ev, st);
        return check_launch(c, "kz_fast");
    }
    KZArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.nx = c->lat.nx;
    a.ny = c->lat.ny;
    a.nz = c->lat.nz;
    a.C = c->C;
    a.yb = c->yb;
    a.j0 = j0;
    a.pz = c->pz;
    a.tw = reinterpret_cast<const cpx<T>*>(c->tw);
    const double pi = 3.14159265358979323846;
    const double lz = c->lat.nz * c->lat.a;
    a.cz = T(2.0 * pi * pi / (lz * lz) / c->lat.nz);
    a.in = in;
    a.G = reinterpret_cast<cpx<T>*>(Gdst);
    dim3 grid(c->lat.ny / c->yb, (unsigned)(k * c->C));
    const size_t lds = kz_lds_bytes(c, c->yb);
    hipEvent_t ev;
    prof_begin(c, 1, &ev, st);
    hipLaunchKernelGGL((kz_kernel<T>), grid, dim3(kThreads), lds, st, a);
    prof_end(c, 1, ev, st);
    return check_launch(c, "kz_kernel");
}

int slots_used(const lise_ctx* c, long long count);

// The single-pass ABM kernel (lise_cube.hpp): the kinetic factors carry
// 1 / N^3 of the 3D round trip.
template <typename T, int N, int MODE>
void launch_kc_n(lise_ctx* c, const KPArgs<T>& a, dim3 grid) {
    if constexpr (cube_side((int)sizeof(T), N)) {
        auto* desc = reinterpret_cast<KPArgs<T>*>(c->cube_desc);
        int* rows = reinterpret_cast<int*>(static_cast<char*>(c->cube_desc) + kDescRowsOffset);
        hipLaunchKernelGGL((put_desc_kernel<T>), dim3(1), dim3(64), 0, c->stream, a, (int)grid.y, desc, rows);
        hipLaunchKernelGGL((kc_fast_batch<T, N, MODE>), grid, dim3(cube_threads_of((int)sizeof(T), N)),
                           cube_lds_of((int)sizeof(T), N), c->stream, desc, rows, 1,
                           reinterpret_cast<const cpx<T>*>(c->tw) + c->tw_full_xy);
    }
}

template <typename T>
void cube_factors(const lise_ctx* c, KPArgs<T>& a) {
    const double pi = 3.14159265358979323846;
    const double n3 = (double)c->N;
    const double lx = c->lat.nx * c->lat.a, ly = c->lat.ny * c->lat.a, lz = c->lat.nz * c->lat.a;
    a.cx = T(2.0 * pi * pi / (lx * lx) / n3);
    a.cy = T(2.0 * pi * pi / (ly * ly) / n3);
    a.cz = T(2.0 * pi * pi / (lz * lz) / n3);
}

template <typename T, int MODE>
int launch_kc_t(lise_ctx* c, KPArgs<T> a, long long j0, int k, int cls) {
    a.j0 = j0;
    a.kcount = k;
    cube_factors<T>(c, a);
    // the kernel reads its descriptor from this device table (written first
    // on the stream); it lives from configure to lise_free
    if (!c->cube_desc) return fail(c, LISE_E_STATE, "single-pass descriptor table is not allocated");
    dim3 grid(1, (unsigned)((k + a.jg - 1) / a.jg));
    hipEvent_t ev;
    prof_begin(c, cls, &ev);
    switch (c->lat.nx) {
        case 8: launch_kc_n<T, 8, MODE>(c, a, grid); break;
        case 16: launch_kc_n<T, 16, MODE>(c, a, grid); break;
        default: launch_kc_n<T, 20, MODE>(c, a, grid); break;
    }
    prof_end(c, cls, ev);
    return check_launch(c, "kc_fast_batch");
}

// One Hamiltonian application over all qpwfs [first, first+count) in chunks:
// z-axis kernel (unless fused) then the plane kernel of the given mode.  With
// overlap on, the z-axis kernel of chunk c+1 runs on the internal stream
// while the plane kernel of chunk c runs on the context stream; the two
// z-scratch buffers alternate and events order every reuse.
// eta_j = <x_j | H | x_j> (Eq. sp_en) for the qpwfs [j0, j0 + k) of the vector
// x = main.in with the fields of `main`; needs the chunk's z-term in main.G.
//
// With the register-FFT kernels on both axes (cheap path) the z kernel of the
// chunk has already written sum_z Re(x^* T_z x) per column into ez (Parseval
// on its forward transform), and the plane pass only needs a forward xy
// transform of x (Parseval again) and the local terms: it reads x alone, not
// the z-term.  Otherwise the plane kernel recomputes H x in full (mode KP_ETA).
bool eta_cheap(const lise_ctx* c) { return c->fast_xy && c->fast_z; }

template <typename T>
int eta_pass_t(lise_ctx* c, const KPArgs<T>& main, long long j0, int k, const double* ez) {
    KPArgs<T> e = main;
    e.jg = 1;
    e.eta = nullptr;
    e.dens_src = 0;
    e.out = e.acc = e.deriv = nullptr;
    e.a1 = e.a2 = e.a3 = e.a4 = e.a5 = e.a6 = nullptr;
    e.epart = c->eta_part;
    const int nblk = plane_grid_x(c);
    const double a3 = c->lat.a * c->lat.a * c->lat.a;
    if (ez) {
        e.jg = kEtaJg;
        CHK((launch_kp_t<T, KP_ETAXY>(c, e, j0, k, 3)));
        const long long nez = (long long)c->C * c->lat.nx * c->lat.ny * c->zl;
        hipLaunchKernelGGL(eta_reduce2_kernel, dim3((unsigned)k), dim3(256), 0, c->stream, c->eta_part,
                           (int)etaxy_parts(c), ez, nez, a3, c->eta + j0);
        return check_launch(c, "eta_reduce2_kernel");
    }
    CHK((launch_kp_t<T, KP_ETA>(c, e, j0, k, 3)));
    hipLaunchKernelGGL(eta_reduce_kernel, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, c->stream, c->eta_part,
                       nblk, k, a3, c->eta + j0);
    return check_launch(c, "eta_reduce_kernel");
}

// eta_op (phase removal of Eq. sp_en, ignored when it is off): 0 plain H;
// 1 compute eta_j of a.in chunk by chunk and apply H - eta_j; 2 apply H - eta_j
// with the eta_j computed by an earlier call.
template <typename T, int MODE>
int apply_chunks(lise_ctx* c, KPArgs<T> a, long long first, long long count, int cls, int eta_op = 0) {
    if (!c->remove_phase) eta_op = 0;
    a.eta = eta_op ? c->eta : nullptr;
    const int dens = a.dens_src;
    if constexpr (MODE == KP_ABM1 || MODE == KP_ABM2) {
        if (c->cube && !a.eta) {   // one pass per chunk, no z-term
            for (long long j0 = first, ci = 0; j0 < first + count; j0 += c->chunk, ++ci) {
                const int k = (int)std::min<long long>(c->chunk, first + count - j0);
                a.G = nullptr;
                a.accumulate = (dens && ci > 0) ? 1 : 0;
                CHK((launch_kc_t<T, MODE>(c, a, j0, k, cls)));
            }
            if (dens && !cube_dens_in_of((int)c->esz / 2, c->lat.nx)) {
                // densities of the vector the phase wrote (m or y_{n+1}) in a
                // pass of their own, into as many slots as the fields kernel sums
                const cpx<T>* v = MODE == KP_ABM1 ? a.a4 : a.a1;
                const long long slots = slots_used(c, c->M);
                const int jgd = (int)((c->M + slots - 1) / slots);
                dim3 grid((unsigned)((c->N + kThreads - 1) / kThreads), (unsigned)slots);
                hipEvent_t ev;
                prof_begin(c, 2, &ev);
                hipLaunchKernelGGL((dens_partial_kernel<T>), grid, dim3(kThreads), 0, c->stream, v, c->C, c->N, c->M,
                                   jgd, c->C == 2 ? c->fn.w : 1.0, c->dpart);
                prof_end(c, 2, ev);
                CHK(check_launch(c, "dens_partial_kernel"));
            }
            return LISE_OK;
        }
        if (c->zdense && !a.eta) {
            // plane kernel only, z-term in the kernel, all qpwfs in one launch
            // (no scratch to size by chunks): ceil(count / jg) density slots
            a.accumulate = 0;
            return launch_kpzd_t<T, MODE>(c, a, first, (int)count, cls);
        }
    }
    const bool ov = c->overlap && !c->fused && c->s2;
    if (ov) {
        HIPCHK(c, hipEventRecord(c->ev_start, c->stream));
        HIPCHK(c, hipStreamWaitEvent(c->s2, c->ev_start, 0));
    }
    const bool cheap = eta_op == 1 && eta_cheap(c);
    for (long long j0 = first, ci = 0; j0 < first + count; j0 += c->chunk, ++ci) {
        const int k = (int)std::min<long long>(c->chunk, first + count - j0);
        const int b = ov ? (int)(ci & 1) : 0;
        void* Gb = c->Gbuf[b];
        double* ez = cheap ? c->ez_part[b] : nullptr;
        if (!c->fused) {
            if (ov) {
                if (ci >= 2) HIPCHK(c, hipStreamWaitEvent(c->s2, c->ev_kp[b], 0));
                CHK(launch_kz_t<T>(c, a.in, j0, k, Gb, c->s2, ez));
                HIPCHK(c, hipEventRecord(c->ev_kz[b], c->s2));
                HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_kz[b], 0));
            } else {
                CHK(launch_kz_t<T>(c, a.in, j0, k, Gb, c->stream, ez));
            }
        }
        a.G = reinterpret_cast<const cpx<T>*>(Gb);
        a.accumulate = (dens && ci > 0) ? 1 : 0;
        if (eta_op == 1) CHK(eta_pass_t<T>(c, a, j0, k, ez));
        CHK((launch_kp_t<T, MODE>(c, a, j0, k, cls)));
        if (ov) HIPCHK(c, hipEventRecord(c->ev_kp[b], c->stream));
    }
    return LISE_OK;
}

int slots_used(const lise_ctx* c, long long count) {
    const long long k = std::min<long long>(c->chunk, count);
    return (int)((k + c->jg - 1) / c->jg);
}

// density slots the ABM phases write: one launch over all qpwfs on the
// in-kernel z-term path, else one chunk's workgroup rows (later chunks add
// into the same slots)
int abm_slots(const lise_ctx* c) {
    return c->zdense ? (int)((c->M + c->jg - 1) / c->jg) : slots_used(c, c->M);
}

// Reduce density partials (nslots > 0) or reuse dens (nslots = 0), optional
// average, then fields at time t.
// toff: time offset from the system's device-side time t_n
int launch_fields(lise_ctx* c, int nslots, const double* avg_with, double* dens, double* V, double* D, double toff) {
    dim3 grid((unsigned)((c->N + kFieldPts - 1) / kFieldPts));
    hipEvent_t ev;
    prof_begin(c, 2, &ev);
    hipLaunchKernelGGL(fields_kernel, grid, dim3(kFieldPts * kFieldGroups), 0, c->stream, c->dpart, nslots, c->N,
                       avg_with, dens, V, D, field_params(c), c->dtime, toff, c->bad);
    prof_end(c, 2, ev);
    return check_launch(c, "fields_kernel");
}

template <typename T>
int dens_direct_t(lise_ctx* c, const cpx<T>* state) {
    const long long slots = (c->M + c->jg - 1) / c->jg;
    dim3 grid((unsigned)((c->N + kThreads - 1) / kThreads), (unsigned)slots);
    hipLaunchKernelGGL((dens_partial_kernel<T>), grid, dim3(kThreads), 0, c->stream, state, c->C, c->N, c->M, c->jg,
                       c->C == 2 ? c->fn.w : 1.0, c->dpart);
    CHK(check_launch(c, "dens_partial_kernel"));
    return launch_fields(c, (int)slots, nullptr, c->dens_cur, c->V_cur, c->D_cur, 0.0);
}

// t_n -> t_n + dt on the device and on the host (the same float64 addition).
int tick(lise_ctx* c, double dt) {
    hipLaunchKernelGGL(tick_kernel, dim3(1), dim3(64), 0, c->stream, c->dtime, dt);
    c->t += dt;
    return check_launch(c, "tick_kernel");
}

int check_bad(lise_ctx* c) {
    int h = 0;
    HIPCHK(c, hipMemcpyAsync(&h, c->bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (h) {
        HIPCHK(c, hipMemsetAsync(c->bad, 0, sizeof(int), c->stream));
        return fail(c, LISE_E_NAN, "non-finite density encountered at t = %g", c->t);
    }
    return LISE_OK;
}

template <typename T>
cpx<T>* ycur(lise_ctx* c) { return S<T>(c, c->iy); }

template <typename T>
int ensure_fields_t(lise_ctx* c) {
    if (c->n_set < c->M) return fail(c, LISE_E_STATE, "qpwfs not fully set (%lld of %lld)", c->n_set, c->M);
    if (!c->dens_valid) {
        CHK(dens_direct_t<T>(c, ycur<T>(c)));
        c->dens_valid = true;
    }
    return LISE_OK;
}

// ---- start-up: series-expansion predictor-corrector -----------------------------

// acc = sum_{q<=4} (-i dt H)^q / q! psi with the fields (V, D); term buffer
// `term`; optional derivative output -i H psi; densities of acc into dpart.
template <typename T>
int taylor_t(lise_ctx* c, const cpx<T>* psi, cpx<T>* term, cpx<T>* acc, cpx<T>* deriv, const double* V,
             const double* D, double dt) {
    for (int q = 1; q <= 4; ++q) {
        KPArgs<T> a = kp_base<T>(c);
        a.V = V;
        a.D = D;
        a.in = (q == 1) ? psi : term;
        a.G = reinterpret_cast<const cpx<T>*>(c->G);
        a.out = term;
        a.acc = acc;
        a.acc_from_in = (q == 1);
        a.deriv = (q == 1) ? deriv : nullptr;
        a.coef_re = 0.0;
        a.coef_im = -dt / q;
        a.dens_src = (q == 4);
        CHK((apply_chunks<T, KP_APPLY>(c, a, 0, c->M, 3, q == 1 ? 1 : 2)));
    }
    return LISE_OK;
}

template <typename T>
int startup_t(lise_ctx* c, double dt) {
    CHK(ensure_fields_t<T>(c));
    // fields of y_0 at t_0
    CHK(launch_fields(c, 0, nullptr, c->dens_cur, c->V_cur, c->D_cur, 0.0));
    int ys = c->iy;             // buffer of Y_s
    const int term = 6;         // p - c slot used as term buffer during start-up
    for (int s = 0; s < 3; ++s) {
        const int acc = 1 - ys;
        // predictor with H(t_s); stores y'_s in derivative slot s
        CHK(taylor_t<T>(c, S<T>(c, ys), S<T>(c, term), S<T>(c, acc), S<T>(c, 2 + s), c->V_cur, c->D_cur, dt));
        // corrector fields from (n_pre + n_s)/2 at t_s + dt/2
        CHK(launch_fields(c, slots_used(c, c->M), c->dens_cur, c->dens_tmp, c->V_tmp, c->D_tmp, 0.5 * dt));
        CHK(taylor_t<T>(c, S<T>(c, ys), S<T>(c, term), S<T>(c, acc), nullptr, c->V_tmp, c->D_tmp, dt));
        CHK(tick(c, dt));
        c->step += 1;
        // densities of Y_{s+1} -> fields at t_{s+1}
        CHK(launch_fields(c, slots_used(c, c->M), nullptr, c->dens_cur, c->V_cur, c->D_cur, 0.0));
        ys = acc;
    }
    // y_n = Y_3 (buffer ys), y_{n-1} = Y_2; derivatives y'_0..y'_2 in slots 0..2
    c->iy = ys;
    c->dn = 3;
    HIPCHK(c, hipMemsetAsync(c->buf[6], 0, (size_t)c->M * c->per * c->esz, c->stream));
    c->hist = true;
    c->dt_hist = dt;
    return check_bad(c);
}

// ---- one ABM step ------------------------------------------------------------------

template <typename T>
int abm_step_t(lise_ctx* c) {
    const double dt = c->dt_hist;
    const int d0 = 2 + c->dn;                   // receives y'_n
    const int d1 = 2 + (c->dn + 3) % 4;         // y'_{n-1}
    const int d2 = 2 + (c->dn + 2) % 4;         // y'_{n-2}
    const int d3 = 2 + (c->dn + 1) % 4;         // y'_{n-3}, then m
    const int yn = c->iy, ym1 = 1 - c->iy;
    // phase 1: H y_n -> y'_n, m, Y; densities of m
    {
        KPArgs<T> a = kp_base<T>(c);
        a.V = c->V_cur;
        a.D = c->D_cur;
        a.in = S<T>(c, yn);
        a.G = reinterpret_cast<const cpx<T>*>(c->G);
        a.a1 = S<T>(c, ym1);
        a.a2 = S<T>(c, d1);
        a.a3 = S<T>(c, d2);
        a.a4 = S<T>(c, d3);
        a.a5 = S<T>(c, 6);
        a.a6 = S<T>(c, d0);
        a.dt = dt;
        a.dens_src = 1;
        CHK((apply_chunks<T, KP_ABM1>(c, a, 0, c->M, 0, 1)));
    }
    CHK(launch_fields(c, abm_slots(c), nullptr, c->dens_tmp, c->V_tmp, c->D_tmp, dt));
    // phase 2: H m -> m', y_{n+1}, p_{n+1} - c_{n+1}; densities of y_{n+1}
    {
        KPArgs<T> a = kp_base<T>(c);
        a.V = c->V_tmp;
        a.D = c->D_tmp;
        a.in = S<T>(c, d3);                         // m
        a.G = reinterpret_cast<const cpx<T>*>(c->G);
        a.a1 = S<T>(c, ym1);                        // Y -> y_{n+1}
        a.a5 = S<T>(c, 6);                          // p_n - c_n -> p_{n+1} - c_{n+1}
        a.dt = dt;
        a.dens_src = 1;
        CHK((apply_chunks<T, KP_ABM2>(c, a, 0, c->M, 4, 1)));
    }
    CHK(launch_fields(c, abm_slots(c), nullptr, c->dens_cur, c->V_cur, c->D_cur, dt));
    CHK(tick(c, dt));
    c->iy = ym1;
    c->dn = (c->dn + 1) % 4;
    c->step += 1;
    return LISE_OK;
}

// Host bookkeeping of one ABM step whose device work ran inside a graph.
void advance_host(lise_ctx* c, double dt) {
    c->t += dt;
    c->iy = 1 - c->iy;
    c->dn = (c->dn + 1) % 4;
    c->step += 1;
}

struct HostState {
    double t;
    long long step;
    int iy, dn;
};
HostState save_host(const lise_ctx* c) { return {c->t, c->step, c->iy, c->dn}; }
void restore_host(lise_ctx* c, const HostState& h) {
    c->t = h.t;
    c->step = h.step;
    c->iy = h.iy;
    c->dn = h.dn;
}

long long ring_sig(const lise_ctx* c) { return (c->config_version * 4 + c->dn) * 2 + c->iy; }

int abm_step_any(lise_ctx* c) { return c->prec == LISE_FP64 ? abm_step_t<double>(c) : abm_step_t<float>(c); }

// Capture kPeriod ABM steps of one system on its current stream (which must
// be capturing).  The ring of buffers returns to its state after kPeriod
// steps, so the captured work can be replayed.  Host bookkeeping is restored.
constexpr int kPeriod = 4;
static_assert(kPeriod == kBatchPeriod, "the batch replays the same ring period");
int capture_period(lise_ctx* c) {
    const HostState h = save_host(c);
    c->capturing = true;
    int rc = LISE_OK;
    for (int i = 0; i < kPeriod && rc == LISE_OK; ++i) rc = abm_step_any(c);
    c->capturing = false;
    restore_host(c, h);
    return rc;
}

int ensure_graph(lise_ctx* c) {
    const long long sig = ring_sig(c);
    if (c->gexec && c->gsig == sig) return LISE_OK;
    if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    // capture on the internal stream (the caller's stream may be the null
    // stream, which cannot be captured); it starts after the caller's work
    HIPCHK(c, hipEventRecord(c->ev_cap, c->stream));
    HIPCHK(c, hipStreamWaitEvent(c->cap, c->ev_cap, 0));
    hipStream_t user = c->stream;
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    c->stream = c->cap;
    int rc = capture_period(c);
    c->stream = user;
    hipError_t e = hipStreamEndCapture(c->cap, &g);
    if (rc != LISE_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(c, LISE_E_HIP, "stream capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(c, LISE_E_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
    c->gsig = sig;
    return LISE_OK;
}

// Enqueue nsteps ABM steps (start-up first when needed) on the context
// stream without waiting for them.
template <typename T>
int advance_t(lise_ctx* c, double dt, long long nsteps) {
    if (!c->hist || c->dt_hist != dt) {
        CHK(startup_t<T>(c, dt));
        if (c->gexec) {
            (void)hipGraphExecDestroy(c->gexec);
            c->gexec = nullptr;
        }
    }
    if (c->use_graph && nsteps >= 2 * kPeriod) {
        CHK(ensure_graph(c));
        for (; nsteps >= kPeriod; nsteps -= kPeriod) {
            HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
            for (int i = 0; i < kPeriod; ++i) advance_host(c, dt);
        }
    }
    for (long long s = 0; s < nsteps; ++s) CHK(abm_step_t<T>(c));
    return LISE_OK;
}

int advance_any(lise_ctx* c, double dt, long long nsteps) {
    return c->prec == LISE_FP64 ? advance_t<double>(c, dt, nsteps) : advance_t<float>(c, dt, nsteps);
}

template <typename T>
int step_t(lise_ctx* c, double dt, long long nsteps) {
    CHK(advance_t<T>(c, dt, nsteps));
    return check_bad(c);
}

// H psi for qpwfs [first, first + count) in pieces of at most kApplyPiece
// bytes of complex128 output: the plane kernel writes a piece (state
// precision) into `stage`, which convert_kernel widens to complex128, straight
// into `out` when it is device memory, else into `stage64` for a copy to the
// host.  stage64 may equal stage in float64.  All buffers are indexed from the
// piece's first qpwf.
constexpr size_t kApplyPiece = 64u << 20;

long long apply_piece_qpwfs(const lise_ctx* c) {
    return std::max<long long>(1, (long long)(kApplyPiece / ((size_t)c->per * sizeof(cpx<double>))));
}

template <typename T>
int apply_pieces_t(lise_ctx* c, long long first, long long count, long long piece, void* stage, void* stage64,
                   void* out, int out_is_device) {
    CHK(ensure_fields_t<T>(c));
    CHK(launch_fields(c, 0, nullptr, c->dens_cur, c->V_cur, c->D_cur, 0.0));
    for (long long j0 = first; j0 < first + count; j0 += piece) {
        const long long k = std::min<long long>(piece, first + count - j0);
        cpx<T>* st = reinterpret_cast<cpx<T>*>(stage);
        KPArgs<T> a = kp_base<T>(c);
        a.V = c->V_cur;
        a.D = c->D_cur;
        a.in = ycur<T>(c);
        a.G = reinterpret_cast<const cpx<T>*>(c->G);
        a.out = st - j0 * c->per;     // the kernel indexes out by the global qpwf
        a.coef_re = 1.0;
        a.coef_im = 0.0;
        a.dens_src = 0;
        CHK((apply_chunks<T, KP_APPLY>(c, a, j0, k, 3)));
        const long long n = k * c->per;
        cpx<double>* dst = out_is_device ? reinterpret_cast<cpx<double>*>(out) + (j0 - first) * c->per
                                         : reinterpret_cast<cpx<double>*>(stage64);
        if (out_is_device || (void*)dst != (void*)st) {
            hipLaunchKernelGGL((convert_kernel<double, T>), dim3(2048), dim3(kThreads), 0, c->stream, st, dst, n);
            CHK(check_launch(c, "convert_kernel"));
        }
        if (!out_is_device) {
            HIPCHK(c, hipMemcpyAsync(reinterpret_cast<cpx<double>*>(out) + (j0 - first) * c->per, dst,
                                     (size_t)n * sizeof(cpx<double>), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));   // stage64 is reused by the next piece
        }
    }
    return LISE_OK;
}

// lise_apply_h: a context-owned staging buffer of one piece (allocated at the
// first call and kept), so that no call allocates more than one piece and
// later calls allocate nothing.
template <typename T>
int apply_h_t(lise_ctx* c, long long first, long long count, void* out, int out_is_device) {
    const long long piece = apply_piece_qpwfs(c);
    const size_t st_bytes = (size_t)piece * c->per * c->esz;
    const size_t need = st_bytes + (sizeof(T) == 8 ? 0 : (size_t)piece * c->per * sizeof(cpx<double>));
    if (c->ah_cap < need) {
        dfree(&c->ah_buf);
        c->ah_cap = 0;
        CHK(dalloc(c, &c->ah_buf, need));
        c->ah_cap = need;
    }
    void* stage = c->ah_buf;
    void* stage64 = sizeof(T) == 8 ? stage : static_cast<char*>(c->ah_buf) + st_bytes;
    return apply_pieces_t<T>(c, first, count, piece, stage, stage64, out, out_is_device);
}

// lise_apply_h_noalloc: the same pieces, staged through this device's fixed
// array (kScratchBytes) instead of the context's buffer; the output is device
// memory, so the piece is widened straight into it.  Allocates nothing.
template <typename T>
int apply_h_noalloc_t(lise_ctx* c, long long first, long long count, void* out) {
    const size_t per_bytes = (size_t)c->per * c->esz;
    if (per_bytes > kScratchBytes)
        return fail(c, LISE_E_UNSUPPORTED, "one qpwf of H psi (%zu bytes) exceeds the %zu-byte fixed staging array",
                    per_bytes, kScratchBytes);
    if (!c->scratch_dev) return fail(c, LISE_E_STATE, "fixed staging array has no device address");
    const long long piece = std::min<long long>(apply_piece_qpwfs(c), (long long)(kScratchBytes / per_bytes));
    return apply_pieces_t<T>(c, first, count, piece, c->scratch_dev, c->scratch_dev, out, 1);
}

// Kinetic energy of the current state (plane kernel in mode KP_KINETIC).  With
// pxy (register-FFT plane kernel only) the same pass also returns the
// Parseval sums of the total current along x and y over the v components:
// pxy[0] = sum m_x |F_xy v|^2, pxy[1] = sum m_y |F_xy v|^2 (signed indices).
template <typename T>
int kinetic_energy_t(lise_ctx* c, double* ekin, double* pxy = nullptr) {
    if (pxy && !c->fast_xy) return fail(c, LISE_E_STATE, "current sums need the register-FFT plane kernel");
    KPArgs<T> a = kp_base<T>(c);
    a.V = c->V_cur;
    a.D = c->D_cur;
    a.in = ycur<T>(c);
    a.G = reinterpret_cast<const cpx<T>*>(c->G);
    const long long nwg_per = (long long)plane_grid_x(c) * ((c->chunk + c->jg - 1) / c->jg);
    const long long need = (pxy ? 3 : 1) * nwg_per;
    if (c->red_cap < need) {
        dfree(reinterpret_cast<void**>(&c->red));
        CHK(dalloc(c, reinterpret_cast<void**>(&c->red), (size_t)std::max<long long>(need, 4096) * sizeof(double)));
        c->red_cap = std::max<long long>(need, 4096);
    }
    a.epart = c->red;
    a.ppart = pxy ? c->red + nwg_per : nullptr;
    std::vector<double> h(need);
    double sum = 0.0, sx = 0.0, sy = 0.0;
    for (long long j0 = 0; j0 < c->M; j0 += c->chunk) {
        const int k = (int)std::min<long long>(c->chunk, c->M - j0);
        if (!c->fused) CHK(launch_kz_t<T>(c, a.in, j0, k, c->Gbuf[0], c->stream));
        a.G = reinterpret_cast<const cpx<T>*>(c->Gbuf[0]);
        CHK((launch_kp_t<T, KP_KINETIC>(c, a, j0, k, 3)));
        const long long nwg = (long long)plane_grid_x(c) * ((k + c->jg - 1) / c->jg);
        HIPCHK(c, hipMemcpyAsync(h.data(), c->red, nwg * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        if (pxy)
            HIPCHK(c, hipMemcpyAsync(h.data() + nwg_per, a.ppart, 2 * nwg * sizeof(double), hipMemcpyDeviceToHost,
                                     c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (long long i = 0; i < nwg; ++i) sum += h[i];
        if (pxy)
            for (long long i = 0; i < nwg; ++i) {
                sx += h[nwg_per + 2 * i];
                sy += h[nwg_per + 2 * i + 1];
            }
    }
    *ekin = sum * c->lat.a * c->lat.a * c->lat.a;
    if (pxy) {
        pxy[0] = sx;
        pxy[1] = sy;
    }
    return LISE_OK;
}

// Parseval sum of the total current along z over the v components,
// sum m_z |F_z v|^2 (register-FFT z kernel only).
template <typename T, int NZ>
void launch_pz_n(const KZFastArgs<T>& f, double* part, unsigned nblk, hipStream_t st) {
    hipLaunchKernelGGL((pz_kernel<T, NZ>), dim3(nblk), dim3(kThreads), 0, st, f, part);
}

template <typename T>
int momentum_z_t(lise_ctx* c, double* pz) {
    if (!c->fast_z) return fail(c, LISE_E_STATE, "z current sum needs the register-FFT z kernel");
    KZFastArgs<T> f;
    std::memset(&f, 0, sizeof(f));
    f.nxy = (long long)c->lat.nx * c->lat.ny;
    f.ncols = c->M * c->C * f.nxy;
    f.j0 = 0;
    f.C = c->C;
    f.tw = reinterpret_cast<const cpx<T>*>(c->tw) + c->tw_full_z;
    f.in = ycur<T>(c);
    f.nu = c->C == 2 ? 1 : 2;
    const long long nblk = (f.ncols + kThreads - 1) / kThreads;
    if (c->pz_cap < nblk) {
        dfree(reinterpret_cast<void**>(&c->pz_part));
        CHK(dalloc(c, reinterpret_cast<void**>(&c->pz_part), (size_t)nblk * sizeof(double)));
        c->pz_cap = nblk;
    }
    switch (c->lat.nz) {
        case 8: launch_pz_n<T, 8>(f, c->pz_part, (unsigned)nblk, c->stream); break;
        case 16: launch_pz_n<T, 16>(f, c->pz_part, (unsigned)nblk, c->stream); break;
        case 20: launch_pz_n<T, 20>(f, c->pz_part, (unsigned)nblk, c->stream); break;
        case 24: launch_pz_n<T, 24>(f, c->pz_part, (unsigned)nblk, c->stream); break;
        case 32: launch_pz_n<T, 32>(f, c->pz_part, (unsigned)nblk, c->stream); break;
        case 48: launch_pz_n<T, 48>(f, c->pz_part, (unsigned)nblk, c->stream); break;
        default: launch_pz_n<T, 64>(f, c->pz_part, (unsigned)nblk, c->stream); break;
    }
    CHK(check_launch(c, "pz_kernel"));
    std::vector<double> h(nblk);
    HIPCHK(c, hipMemcpyAsync(h.data(), c->pz_part, nblk * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double s = 0.0;
    for (long long i = 0; i < nblk; ++i) s += h[i];
    *pz = s;
    return LISE_OK;
}

template <typename T>
int norms_t(lise_ctx* c, double* dst) {
    hipLaunchKernelGGL((norm_kernel<T>), dim3((unsigned)c->M), dim3(kThreads), 0, c->stream, ycur<T>(c), c->per, dst);
    return check_launch(c, "norm_kernel");
}

template <typename T, int NS>
void launch_jx_n(const CurArgs<T>& a, const cpx<T>* twN, int nslots, hipStream_t st) {
    hipLaunchKernelGGL((jx_fast<T, NS>), dim3(a.nz, nslots), dim3(plane_block<T, NS>()), 0, st, a, twN);
}

template <typename T, int NA>
void launch_jline_n(const CurArgs<T>& a, const cpx<T>* tw, int nslots, long long nlines, long long inner,
                    long long outer, long long es, T f, int axis, hipStream_t st) {
    dim3 grid((unsigned)((nlines + kJLineThreads - 1) / kJLineThreads), nslots);
    hipLaunchKernelGGL((jline_fast<T, NA>), grid, dim3(kJLineThreads), 0, st, a, tw, nlines, inner, outer, es, f, axis);
}

// lines of a side n <= 32 along one axis (register FFTs)
template <typename T>
void launch_jline(const CurArgs<T>& a, int n, const cpx<T>* tw, int nslots, long long nlines, long long inner,
                  long long outer, long long es, T f, int axis, hipStream_t st) {
    switch (n) {
        case 8: launch_jline_n<T, 8>(a, tw, nslots, nlines, inner, outer, es, f, axis, st); break;
        case 16: launch_jline_n<T, 16>(a, tw, nslots, nlines, inner, outer, es, f, axis, st); break;
        case 20: launch_jline_n<T, 20>(a, tw, nslots, nlines, inner, outer, es, f, axis, st); break;
        case 24: launch_jline_n<T, 24>(a, tw, nslots, nlines, inner, outer, es, f, axis, st); break;
        default: launch_jline_n<T, 32>(a, tw, nslots, nlines, inner, outer, es, f, axis, st); break;
    }
}

// Current density of Eq. (j) of the current state into jdev (3N float64: x, y, z).
// Register-FFT kernels where both plane and z kernels have them and the sides
// are at most 32; LDS Stockham kernels otherwise.
template <typename T>
int current_t(lise_ctx* c, double* jdev) {
    const int nx = c->lat.nx, ny = c->lat.ny, nz = c->lat.nz;
    const long long nxy = (long long)nx * ny;
    const bool fast = c->fast_xy && c->fast_z && nx <= 32 && nz <= 32;
    const int cap = c->prec == LISE_FP64 ? 2048 : 4096;
    int yb = 0;
    for (int d = ny; d >= 1; --d)
        if (ny % d == 0 && (long long)d * nx * nz <= cap) { yb = d; break; }
    const size_t lds_xy = 2 * (size_t)nxy * c->esz;
    const size_t lds_z = 2 * (size_t)nz * yb * nx * c->esz;
    if (!fast && (nxy > 16 * kThreads || yb == 0 || lds_xy > c->lds_limit || lds_z > c->lds_limit))
        return fail(c, LISE_E_UNSUPPORTED, "current density: lattice %dx%dx%d too large for the LDS kernels", nx, ny, nz);
    CurArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.C = c->C;
    a.yb = yb;
    a.jg = c->jg;
    a.M = c->M;
    a.nv = c->C == 2 ? 1 : 2;
    a.v0 = c->C == 2 ? 1 : 2;
    a.w = c->C == 2 ? c->fn.w : 1.0;
    a.px = c->px;
    a.py = c->py;
    a.pz = c->pz;
    a.tw = reinterpret_cast<const cpx<T>*>(c->tw);
    const double pi = 3.14159265358979323846;
    a.fx = T(2.0 * pi / (nx * c->lat.a) / nx);
    a.fy = T(2.0 * pi / (ny * c->lat.a) / ny);
    a.fz = T(2.0 * pi / (nz * c->lat.a) / nz);
    a.in = ycur<T>(c);
    a.jpart = c->dpart;
    const int nslots = (int)((c->M + c->jg - 1) / c->jg);
    if (nslots > c->slot_cap) return fail(c, LISE_E_STATE, "partial-sum buffer too small");
    if (fast) {
        const cpx<T>* twxy = reinterpret_cast<const cpx<T>*>(c->tw) + c->tw_full_xy;
        const cpx<T>* twz = reinterpret_cast<const cpx<T>*>(c->tw) + c->tw_full_z;
        switch (nx) {
            case 8: launch_jx_n<T, 8>(a, twxy, nslots, c->stream); break;
            case 16: launch_jx_n<T, 16>(a, twxy, nslots, c->stream); break;
            case 20: launch_jx_n<T, 20>(a, twxy, nslots, c->stream); break;
            case 24: launch_jx_n<T, 24>(a, twxy, nslots, c->stream); break;
            default: launch_jx_n<T, 32>(a, twxy, nslots, c->stream); break;
        }
        CHK(check_launch(c, "jx_fast"));
        // y lines: line t = (z, x), points nx apart (nx == ny on this path)
        launch_jline<T>(a, ny, twxy, nslots, (long long)nx * nz, nx, nxy, nx, a.fy, 1, c->stream);
        CHK(check_launch(c, "jline_fast y"));
        // z lines: line t = xy point, points nxy apart
        launch_jline<T>(a, nz, twz, nslots, nxy, nxy, 0, nxy, a.fz, 2, c->stream);
        CHK(check_launch(c, "jline_fast z"));
    } else {
        const long long pz = (long long)nz * yb * nx;
        if (nxy <= 4 * kThreads)
            hipLaunchKernelGGL((current_xy_kernel<T, 4>), dim3(nz, nslots), dim3(kThreads), lds_xy, c->stream, a);
        else
            hipLaunchKernelGGL((current_xy_kernel<T, 16>), dim3(nz, nslots), dim3(kThreads), lds_xy, c->stream, a);
        CHK(check_launch(c, "current_xy_kernel"));
        if (pz <= 4 * kThreads)
            hipLaunchKernelGGL((current_z_kernel<T, 4>), dim3(ny / yb, nslots), dim3(kThreads), lds_z, c->stream, a);
        else
            hipLaunchKernelGGL((current_z_kernel<T, 16>), dim3(ny / yb, nslots), dim3(kThreads), lds_z, c->stream, a);
        CHK(check_launch(c, "current_z_kernel"));
    }
    const long long n3 = 3 * c->N;
    hipLaunchKernelGGL(slot_sum_kernel, dim3((unsigned)((n3 + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       c->stream, c->dpart, nslots, n3, jdev);
    return check_launch(c, "slot_sum_kernel");
}

// Eq. (kick) on the current state; chi is a device array of N float64.
template <typename T>
int kick_t(lise_ctx* c, const double* chi_dev) {
    double* phase = c->dens_tmp;   // 2N of its 3N doubles: scratch between steps
    hipLaunchKernelGGL(phase_kernel, dim3((unsigned)((c->N + kThreads - 1) / kThreads)), dim3(kThreads), 0, c->stream,
                       chi_dev, c->N, phase);
    CHK(check_launch(c, "phase_kernel"));
    const long long total = c->M * c->per;
    hipLaunchKernelGGL((kick_kernel<T>), dim3(4096), dim3(kThreads), 0, c->stream, ycur<T>(c), phase, c->N, c->C,
                       c->C == 2 ? 1 : 2, total);
    return check_launch(c, "kick_kernel");
}

template <typename T>
int observables_t(lise_ctx* c, lise_obs* o) {
    CHK(ensure_fields_t<T>(c));
    CHK(launch_fields(c, 0, nullptr, c->dens_cur, c->V_cur, c->D_cur, 0.0));
    const int nblk = 256;
    if (c->red_cap < nblk * kNObs) {
        dfree(reinterpret_cast<void**>(&c->red));
        CHK(dalloc(c, reinterpret_cast<void**>(&c->red), 4096 * sizeof(double)));
        c->red_cap = 4096;
    }
    hipLaunchKernelGGL(obs_fields_kernel, dim3(nblk), dim3(kThreads), 0, c->stream, c->dens_cur, c->D_cur, c->N,
                       field_params(c), c->t, c->red);
    CHK(check_launch(c, "obs_fields_kernel"));
    std::vector<double> h(nblk * kNObs);
    HIPCHK(c, hipMemcpyAsync(h.data(), c->red, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double s[kNObs] = {0};
    for (int b = 0; b < nblk; ++b)
        for (int k = 0; k < kNObs; ++k) s[k] += h[b * kNObs + k];
    double ekin = 0.0;
    // with the register-FFT kernels on both axes the total current comes from
    // Parseval sums (the kinetic pass gives x and y, one more pass over the v
    // components z) instead of the current-density field
    const bool parseval_p = c->fast_xy && c->fast_z;
    double pxy[2] = {0.0, 0.0};
    CHK(kinetic_energy_t<T>(c, &ekin, parseval_p ? pxy : nullptr));
    const double a3 = c->lat.a * c->lat.a * c->lat.a;
    std::memset(o, 0, sizeof(*o));
    o->t = c->t;
    o->step = c->step;
    o->N = a3 * s[0];
    o->E_kin = ekin;
    o->E_int = a3 * s[4];
    o->E_pair = a3 * s[5];
    o->E_ext = a3 * s[6];
    o->E = o->E_kin + o->E_int + o->E_pair + o->E_ext;
    o->mean_abs_delta = s[0] != 0.0 ? s[7] / s[0] : 0.0;
    for (int k = 0; k < 3; ++k) o->r_cm[k] = s[0] != 0.0 ? s[1 + k] / s[0] : 0.0;
    // norm drift
    CHK(norms_t<T>(c, c->norms));
    std::vector<double> n1(c->M), n0(c->M);
    HIPCHK(c, hipMemcpyAsync(n1.data(), c->norms, c->M * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(n0.data(), c->norms0, c->M * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double mx = 0.0, mean = 0.0;
    for (long long j = 0; j < c->M; ++j) {
        const double d = std::fabs(n1[j] - n0[j]) * a3;
        mx = std::max(mx, d);
        mean += d;
    }
    o->norm_drift_max = mx;
    o->norm_drift_mean = c->M ? mean / c->M : 0.0;
    // spin-resolved numbers (Eq. rho_t): C = 4 sums |v_up|^2 and |v_dn|^2 per
    // qpwf; the C = 2 reduction is spin-symmetric
    if (c->C == 4) {
        double* part = c->dens_tmp;   // 2M doubles of scratch between steps
        if (2 * c->M > 3 * c->N) {
            if (c->red_cap < 2 * c->M) {
                dfree(reinterpret_cast<void**>(&c->red));
                CHK(dalloc(c, reinterpret_cast<void**>(&c->red), (size_t)(2 * c->M) * sizeof(double)));
                c->red_cap = 2 * c->M;
            }
            part = c->red;
        }
        hipLaunchKernelGGL((comp_norm_kernel<T>), dim3((unsigned)(2 * c->M)), dim3(kThreads), 0, c->stream, ycur<T>(c),
                           c->C, 2, 2, c->N, part);
        CHK(check_launch(c, "comp_norm_kernel"));
        std::vector<double> hs(2 * c->M);
        HIPCHK(c, hipMemcpyAsync(hs.data(), part, hs.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        double up = 0.0, dn = 0.0;
        for (long long j = 0; j < c->M; ++j) {
            up += hs[2 * j];
            dn += hs[2 * j + 1];
        }
        o->N_up = a3 * up;
        o->N_dn = a3 * dn;
    } else {
        o->N_up = o->N_dn = 0.5 * o->N;
    }
    // total current and centre-of-mass velocity (Eq. j, Eq. vel with m = hbar = 1)
    if (parseval_p) {
        // sum_r Im(v^* d_a v) = (2 pi / L_a) sum_k m_a |F v|^2 / (transform size):
        // the xy sums come from 2D transforms of the planes, the z sum from 1D
        // transforms of the columns
        double sz = 0.0;
        CHK(momentum_z_t<T>(c, &sz));
        const double pi = 3.14159265358979323846;
        const double w = c->C == 2 ? c->fn.w : 1.0;
        const double nxy = (double)c->lat.nx * c->lat.ny;
        o->P[0] = -w * a3 * (2.0 * pi / (c->lat.nx * c->lat.a)) * pxy[0] / nxy;
        o->P[1] = -w * a3 * (2.0 * pi / (c->lat.ny * c->lat.a)) * pxy[1] / nxy;
        o->P[2] = -w * a3 * (2.0 * pi / (c->lat.nz * c->lat.a)) * sz / c->lat.nz;
    } else {
        CHK(current_t<T>(c, c->dens_tmp));
        std::vector<double> jh(3 * c->N);
        HIPCHK(c, hipMemcpyAsync(jh.data(), c->dens_tmp, jh.size() * sizeof(double), hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int k = 0; k < 3; ++k) {
            double sum = 0.0;
            for (long long r = 0; r < c->N; ++r) sum += jh[k * c->N + r];
            o->P[k] = a3 * sum;
        }
    }
    for (int k = 0; k < 3; ++k) o->v_cm[k] = o->N != 0.0 ? o->P[k] / o->N : 0.0;
    return LISE_OK;
}

// Forget which qpwfs were written (they must all be set again).
void reset_coverage(lise_ctx* c) {
    std::fill(c->set_mask.begin(), c->set_mask.end(), (unsigned char)0);
    c->n_set = 0;
}

int valid_dim(int n) {
    if (n < 1 || n > 128) return 0;
    int m = n;
    for (int p : {2, 3, 5})
        while (m % p == 0) m /= p;
    return m == 1;
}

}  // namespace

// A batch of independent systems advanced together.  Systems whose lattice
// the register-FFT kernels cover are grouped by (precision, xy side, z side);
// per ABM phase each group runs ONE z-axis launch and ONE plane-kernel launch
// over all qpwfs of all its systems, driven by device tables with one
// descriptor per system (its buffers, fields, functional, qpwf count).  One
// launch reduces the densities and forms the fields of every system, one more
// advances every system's time.  Four steps (one period of the buffer ring)
// are captured once, on a single internal stream, as one graph holding only
// kernel nodes, and replayed.  Other systems step one after another on the
// batch stream.
struct BatchGroup {
    int prec = LISE_FP64;
    int nx = 0, nz = 0;
    bool cube = false;             // single-pass kernel, no z-axis launch or z-scratch
    bool dens_split = false;       // single-pass kernel without densities: a density pass follows
    int zl = 1;                    // lanes per z-column
    long long dblocks = 0;         // workgroups of the density pass
    size_t off_dblks = 0;
    size_t off_dens[kBatchPeriod][2] = {};
    std::vector<int> sys;          // indices into lise_batch::sys
    std::vector<size_t> goff;      // byte offset of each system's region of the z-scratch
    size_t gbytes = 0;             // z-scratch of the group: sum of M * C * N elements
    long long qpwfs = 0;           // sum of M over the group
    int rows = 0;                  // plane-kernel workgroup rows (sum of ceil(M / jg))
    long long zblocks = 0;         // z-kernel workgroups
    size_t off_rows = 0, off_blks = 0;   // device table offsets (bytes)
    size_t off_kp[kBatchPeriod][2] = {}, off_kz[kBatchPeriod][2] = {};
};

struct lise_batch {
    std::vector<lise_ctx*> sys;
    hipStream_t stream = nullptr;   // caller's stream (may be the null stream)
    hipStream_t cap = nullptr;      // internal stream the graph is captured on
    hipEvent_t ev_cap = nullptr;
    std::vector<BatchGroup> groups;
    std::vector<int> grouped, solo;   // systems in a group / stepped one by one
    void* G = nullptr;               // z-scratch of the largest group
    size_t g_bytes = 0;
    void* dtab = nullptr;            // descriptor tables
    size_t dtab_bytes = 0;
    size_t off_fblks = 0, off_fd[2] = {0, 0}, off_tick = 0;
    long long fblocks = 0;
    bool tables = false;
    double tab_dt = 0.0;
    int tphase = 0;                  // steps taken since the tables' base ring state
    std::vector<int> base_iy, base_dn;
    std::vector<long long> base_cfg;
    int use_graph = 1;
    hipGraphExec_t gexec = nullptr;
    Prof prof;
    char err[512] = {0};
};

namespace {

int bfail(lise_batch* b, int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(b->err, sizeof(b->err), fmt, ap);
    va_end(ap);
    return code;
}

#define BCHK(call)                 \
    do {                           \
        int rc_ = (call);          \
        if (rc_ != LISE_OK) return rc_; \
    } while (0)

int bcheck_launch(lise_batch* b, const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return bfail(b, LISE_E_HIP, "launch of %s failed: %s", what, hipGetErrorString(e));
    return LISE_OK;
}

// per-class event pairs around the batch's launches (0 plane kernel of phase 1,
// 1 z axis, 2 fields, 3 plane kernel of phase 2)
void bprof_begin(lise_batch* b, hipEvent_t* ev, hipStream_t st) {
    *ev = nullptr;
    if (!b->prof.on) return;
    if (b->prof.used + 2 > b->prof.pool.size()) {
        b->prof.overflow = true;
        return;
    }
    *ev = b->prof.pool[b->prof.used];
    (void)hipEventRecord(*ev, st);
}
void bprof_end(lise_batch* b, int cls, hipEvent_t a, hipStream_t st) {
    if (!a) return;
    hipEvent_t e = b->prof.pool[b->prof.used + 1];
    b->prof.used += 2;
    (void)hipEventRecord(e, st);
    b->prof.recs.push_back({cls, a, e});
}

// A system joins a group when both register-FFT kernels cover its lattice and
// no per-qpwf pass (phase removal) or other plane kernel is in use.
bool batch_groupable(const lise_ctx* c) {
    return c->fast_xy && c->fast_z && !c->mfma_xy && !c->fused && !c->remove_phase && !c->generic && !c->zdense;
}

// slots and slot width of the separate density pass (as apply_chunks)
long long split_slots(const lise_ctx* c) { return slots_used(c, c->M); }
int split_jgd(const lise_ctx* c) { return (int)((c->M + split_slots(c) - 1) / split_slots(c)); }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Ring state of system c after `step` steps from the tables' base state.
void batch_ring(const lise_batch* b, int i, int step, int* iy, int* dn) {
    *iy = b->base_iy[i] ^ (step & 1);
    *dn = (b->base_dn[i] + step) % 4;
}

template <typename T>
void batch_fill_group(lise_batch* b, const BatchGroup& g, std::vector<unsigned char>& h, double dt) {
    const int ns = (int)g.sys.size();
    std::vector<int> rows(ns + 1, 0);
    std::vector<long long> blks(ns + 1, 0);
    for (int i = 0; i < ns; ++i) {
        const lise_ctx* c = b->sys[g.sys[i]];
        rows[i + 1] = rows[i] + (int)((c->M + c->jg - 1) / c->jg);
        const long long ncols = c->M * c->C * (long long)c->lat.nx * c->lat.ny;
        blks[i + 1] = blks[i] + (ncols * c->zl + kThreads - 1) / kThreads;
    }
    std::memcpy(h.data() + g.off_rows, rows.data(), rows.size() * sizeof(int));
    std::memcpy(h.data() + g.off_blks, blks.data(), blks.size() * sizeof(long long));
    std::vector<long long> dblks(ns + 1, 0);
    for (int i = 0; i < ns; ++i) {
        const lise_ctx* c = b->sys[g.sys[i]];
        dblks[i + 1] = dblks[i] + split_slots(c) * ((c->N + kThreads - 1) / kThreads);
    }
    std::memcpy(h.data() + g.off_dblks, dblks.data(), dblks.size() * sizeof(long long));
    for (int st = 0; st < kBatchPeriod; ++st)
        for (int ph = 0; ph < 2; ++ph)
            for (int i = 0; i < ns; ++i) {
                lise_ctx* c = b->sys[g.sys[i]];
                int iy, dn;
                batch_ring(b, g.sys[i], st, &iy, &dn);
                const int d0 = 2 + dn, d1 = 2 + (dn + 3) % 4, d2 = 2 + (dn + 2) % 4, d3 = 2 + (dn + 1) % 4;
                const int yn = iy, ym1 = 1 - iy;
                cpx<T>* Gs = g.cube ? nullptr : reinterpret_cast<cpx<T>*>(static_cast<char*>(b->G) + g.goff[i]);
                KPArgs<T> a = kp_base<T>(c);
                a.j0 = 0;
                a.kcount = (int)c->M;
                a.G = g.cube ? nullptr : Gs;
                if (g.cube) cube_factors<T>(c, a);
                a.dt = dt;
                a.dens_src = 1;
                a.accumulate = 0;
                a.eta = nullptr;
                if (ph == 0) {   // as abm_step_t, phase 1
                    a.V = c->V_cur;
                    a.D = c->D_cur;
                    a.in = S<T>(c, yn);
                    a.a1 = S<T>(c, ym1);
                    a.a2 = S<T>(c, d1);
                    a.a3 = S<T>(c, d2);
                    a.a4 = S<T>(c, d3);
                    a.a5 = S<T>(c, 6);
                    a.a6 = S<T>(c, d0);
                } else {         // phase 2
                    a.V = c->V_tmp;
                    a.D = c->D_tmp;
                    a.in = S<T>(c, d3);
                    a.a1 = S<T>(c, ym1);
                    a.a5 = S<T>(c, 6);
                }
                std::memcpy(h.data() + g.off_kp[st][ph] + i * sizeof(KPArgs<T>), &a, sizeof(a));
                KZFastArgs<T> f;
                std::memset(&f, 0, sizeof(f));
                f.nxy = (long long)c->lat.nx * c->lat.ny;
                f.ncols = c->M * c->C * f.nxy;
                f.j0 = 0;
                f.C = c->C;
                const double pi = 3.14159265358979323846;
                const double lz = c->lat.nz * c->lat.a;
                f.cz = T(2.0 * pi * pi / (lz * lz) / c->lat.nz);
                f.tw = reinterpret_cast<const cpx<T>*>(c->tw) + c->tw_full_z;
                f.in = a.in;
                f.G = Gs;
                f.ezpart = nullptr;
                f.nu = c->C == 2 ? 1 : 2;
                std::memcpy(h.data() + g.off_kz[st][ph] + i * sizeof(KZFastArgs<T>), &f, sizeof(f));
                DensDesc<T> dd;
                std::memset(&dd, 0, sizeof(dd));
                dd.v = ph == 0 ? a.a4 : a.a1;   // m, or y_{n+1}
                dd.N = c->N;
                dd.M = c->M;
                dd.C = c->C;
                dd.jgd = split_jgd(c);
                dd.w = c->C == 2 ? c->fn.w : 1.0;
                dd.dpart = c->dpart;
                dd.bx = (c->N + kThreads - 1) / kThreads;
                std::memcpy(h.data() + g.off_dens[st][ph] + i * sizeof(DensDesc<T>), &dd, sizeof(dd));
            }
}

// (Re)build the groups, the z-scratch and the descriptor tables for the
// systems' current ring states.
int batch_build(lise_batch* b, double dt) {
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    b->tables = false;
    b->groups.clear();
    b->grouped.clear();
    b->solo.clear();
    const int ns = (int)b->sys.size();
    for (int i = 0; i < ns; ++i) {
        lise_ctx* c = b->sys[i];
        if (!batch_groupable(c)) {
            b->solo.push_back(i);
            continue;
        }
        BatchGroup* g = nullptr;
        for (auto& x : b->groups)
            if (x.prec == c->prec && x.nx == c->lat.nx && x.nz == c->lat.nz && x.cube == c->cube && x.zl == c->zl)
                g = &x;
        if (!g) {
            b->groups.emplace_back();
            g = &b->groups.back();
            g->prec = c->prec;
            g->nx = c->lat.nx;
            g->nz = c->lat.nz;
            g->cube = c->cube;
            g->dens_split = c->cube && !cube_dens_in_of((int)c->esz / 2, c->lat.nx);
            g->zl = c->zl;
        }
        g->sys.push_back(i);
        g->goff.push_back(g->gbytes);   // systems of one group may differ in C
        if (!c->cube) g->gbytes += (size_t)c->M * c->per * c->esz;
        g->qpwfs += c->M;
        g->rows += (int)((c->M + c->jg - 1) / c->jg);
        g->zblocks += (c->M * c->C * (long long)c->lat.nx * c->lat.ny * c->zl + kThreads - 1) / kThreads;
        g->dblocks += split_slots(c) * ((c->N + kThreads - 1) / kThreads);
        b->grouped.push_back(i);
    }
    if (b->grouped.empty()) return LISE_OK;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return bfail(b, LISE_E_HIP, "device properties");
    size_t gneed = 0;
    for (auto& g : b->groups) {
        if (g.rows > prop.maxGridSize[1])
            return bfail(b, LISE_E_UNSUPPORTED, "group %dx%dx%d: %d workgroup rows exceed the grid limit %d", g.nx, g.nx,
                         g.nz, g.rows, prop.maxGridSize[1]);
        gneed = std::max(gneed, g.gbytes);
    }
    if (b->g_bytes < gneed) {
        dfree(&b->G);
        b->g_bytes = 0;
        if (hipMalloc(&b->G, gneed) != hipSuccess) {
            b->G = nullptr;
            return bfail(b, LISE_E_NOMEM, "batch z-scratch of %zu bytes", gneed);
        }
        b->g_bytes = gneed;
    }
    // table layout
    size_t off = 0;
    for (auto& g : b->groups) {
        const size_t n = g.sys.size();
        const size_t kp_sz = g.prec == LISE_FP64 ? sizeof(KPArgs<double>) : sizeof(KPArgs<float>);
        const size_t kz_sz = g.prec == LISE_FP64 ? sizeof(KZFastArgs<double>) : sizeof(KZFastArgs<float>);
        g.off_rows = off;
        off = align256(off + (n + 1) * sizeof(int));
        g.off_blks = off;
        off = align256(off + (n + 1) * sizeof(long long));
        g.off_dblks = off;
        off = align256(off + (n + 1) * sizeof(long long));
        const size_t dd_sz = g.prec == LISE_FP64 ? sizeof(DensDesc<double>) : sizeof(DensDesc<float>);
        for (int st = 0; st < kBatchPeriod; ++st)
            for (int ph = 0; ph < 2; ++ph) {
                g.off_kp[st][ph] = off;
                off = align256(off + n * kp_sz);
                g.off_kz[st][ph] = off;
                off = align256(off + n * kz_sz);
                g.off_dens[st][ph] = off;
                off = align256(off + n * dd_sz);
            }
    }
    const size_t ng = b->grouped.size();
    b->off_fblks = off;
    off = align256(off + (ng + 1) * sizeof(long long));
    for (int ph = 0; ph < 2; ++ph) {
        b->off_fd[ph] = off;
        off = align256(off + ng * sizeof(FieldsDesc));
    }
    b->off_tick = off;
    off = align256(off + ng * sizeof(double*));
    if (b->dtab_bytes < off) {
        dfree(&b->dtab);
        b->dtab_bytes = 0;
        if (hipMalloc(&b->dtab, off) != hipSuccess) {
            b->dtab = nullptr;
            return bfail(b, LISE_E_NOMEM, "batch tables of %zu bytes", off);
        }
        b->dtab_bytes = off;
    }
    b->base_iy.assign(ns, 0);
    b->base_dn.assign(ns, 0);
    b->base_cfg.assign(ns, 0);
    for (int i = 0; i < ns; ++i) {
        b->base_iy[i] = b->sys[i]->iy;
        b->base_dn[i] = b->sys[i]->dn;
        b->base_cfg[i] = b->sys[i]->config_version;
    }
    std::vector<unsigned char> h(off, 0);
    for (auto& g : b->groups) {
        if (g.prec == LISE_FP64) batch_fill_group<double>(b, g, h, dt);
        else batch_fill_group<float>(b, g, h, dt);
    }
    std::vector<long long> fb(ng + 1, 0);
    std::vector<double*> tk(ng, nullptr);
    for (size_t k = 0; k < ng; ++k) {
        lise_ctx* c = b->sys[b->grouped[k]];
        fb[k + 1] = fb[k] + (c->N + kFieldPts - 1) / kFieldPts;
        tk[k] = c->dtime;
        for (int ph = 0; ph < 2; ++ph) {
            FieldsDesc d;
            std::memset(&d, 0, sizeof(d));
            d.dpart = c->dpart;
            // the slots the plane or single-pass kernel writes (one per workgroup
            // row), or those of the separate density pass
            d.nslots = (c->cube && !cube_dens_in_of((int)c->esz / 2, c->lat.nx)) ? (int)split_slots(c)
                                                                               : (int)((c->M + c->jg - 1) / c->jg);
            d.N = c->N;
            d.dens = ph == 0 ? c->dens_tmp : c->dens_cur;
            d.V = ph == 0 ? c->V_tmp : c->V_cur;
            d.D = ph == 0 ? c->D_tmp : c->D_cur;
            d.fp = field_params(c);
            d.tdev = c->dtime;
            d.bad = c->bad;
            std::memcpy(h.data() + b->off_fd[ph] + k * sizeof(FieldsDesc), &d, sizeof(d));
        }
    }
    b->fblocks = fb[ng];
    std::memcpy(h.data() + b->off_fblks, fb.data(), fb.size() * sizeof(long long));
    std::memcpy(h.data() + b->off_tick, tk.data(), tk.size() * sizeof(double*));
    // the batch stream may still run earlier steps that read the old tables
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e == hipSuccess) e = hipMemcpy(b->dtab, h.data(), off, hipMemcpyHostToDevice);
    if (e != hipSuccess) return bfail(b, LISE_E_HIP, "batch tables: %s", hipGetErrorString(e));
    b->tables = true;
    b->tab_dt = dt;
    b->tphase = 0;
    return LISE_OK;
}

// Whether the tables still describe every grouped system: same tuning, dt,
// and each ring advanced by exactly tphase steps from the base.
bool batch_tables_valid(const lise_batch* b, double dt) {
    if (!b->tables || b->tab_dt != dt) return false;
    for (int i : b->grouped) {
        const lise_ctx* c = b->sys[i];
        int iy, dn;
        batch_ring(b, i, b->tphase, &iy, &dn);
        if (c->config_version != b->base_cfg[i] || c->iy != iy || c->dn != dn || !batch_groupable(c)) return false;
    }
    for (int i : b->solo)
        if (batch_groupable(b->sys[i])) return false;
    return true;
}

template <typename T, int MODE, int NS>
void launch_kp_batch_n(lise_batch* b, const BatchGroup& g, int st, const cpx<T>* twN, hipStream_t s) {
    constexpr int block = plane_block<T, NS>();
    const size_t lds = std::max(kp_fast_lds<T, NS>(), (size_t)block * sizeof(double));
    const char* base = static_cast<const char*>(b->dtab);
    const auto* tab = reinterpret_cast<const KPArgs<T>*>(base + g.off_kp[st][MODE == KP_ABM1 ? 0 : 1]);
    const auto* rows = reinterpret_cast<const int*>(base + g.off_rows);
    hipLaunchKernelGGL((kp_fast_batch<T, NS, MODE>), dim3((unsigned)g.nz, (unsigned)g.rows), dim3(block), lds, s, tab,
                       rows, (int)g.sys.size(), twN);
}

template <typename T, int MODE, int NS>
void launch_kc_batch_n(lise_batch* b, const BatchGroup& g, int st, const cpx<T>* twN, hipStream_t s) {
    if constexpr (cube_side((int)sizeof(T), NS)) {
        const char* base = static_cast<const char*>(b->dtab);
        const auto* tab = reinterpret_cast<const KPArgs<T>*>(base + g.off_kp[st][MODE == KP_ABM1 ? 0 : 1]);
        const auto* rows = reinterpret_cast<const int*>(base + g.off_rows);
        hipLaunchKernelGGL((kc_fast_batch<T, NS, MODE>), dim3(1, (unsigned)g.rows),
                           dim3(cube_threads_of((int)sizeof(T), NS)), cube_lds_of((int)sizeof(T), NS), s, tab, rows,
                           (int)g.sys.size(), twN);
    }
}

template <typename T, int MODE>
int launch_kp_batch(lise_batch* b, const BatchGroup& g, int st, hipStream_t s) {
    const lise_ctx* c0 = b->sys[g.sys[0]];
    const cpx<T>* twN = reinterpret_cast<const cpx<T>*>(c0->tw) + c0->tw_full_xy;
    hipEvent_t ev;
    bprof_begin(b, &ev, s);
    if (g.cube) {
        switch (g.nx) {
            case 8: launch_kc_batch_n<T, MODE, 8>(b, g, st, twN, s); break;
            case 16: launch_kc_batch_n<T, MODE, 16>(b, g, st, twN, s); break;
            default: launch_kc_batch_n<T, MODE, 20>(b, g, st, twN, s); break;
        }
        bprof_end(b, MODE == KP_ABM1 ? 0 : 3, ev, s);
        return bcheck_launch(b, "kc_fast_batch");
    }
    switch (g.nx) {
        case 8: launch_kp_batch_n<T, MODE, 8>(b, g, st, twN, s); break;
        case 16: launch_kp_batch_n<T, MODE, 16>(b, g, st, twN, s); break;
        case 20: launch_kp_batch_n<T, MODE, 20>(b, g, st, twN, s); break;
        case 24: launch_kp_batch_n<T, MODE, 24>(b, g, st, twN, s); break;
        case 32: launch_kp_batch_n<T, MODE, 32>(b, g, st, twN, s); break;
        case 48: launch_kp_batch_n<T, MODE, 48>(b, g, st, twN, s); break;
        default: launch_kp_batch_n<T, MODE, 64>(b, g, st, twN, s); break;
    }
    bprof_end(b, MODE == KP_ABM1 ? 0 : 3, ev, s);
    return bcheck_launch(b, "kp_fast_batch");
}

template <typename T, int NZ, int L>
void launch_kz_batch_l(lise_batch* b, const BatchGroup& g, int st, int ph, bool nt, hipStream_t s) {
    if constexpr (kz_lanes_valid(NZ, L)) {
        const char* base = static_cast<const char*>(b->dtab);
        const auto* tab = reinterpret_cast<const KZFastArgs<T>*>(base + g.off_kz[st][ph]);
        const auto* blks = reinterpret_cast<const long long*>(base + g.off_blks);
        const dim3 grid((unsigned)g.zblocks);
        if (nt)
            hipLaunchKernelGGL((kz_fast_batch<T, NZ, L, true>), grid, dim3(kThreads), 0, s, tab, blks,
                               (int)g.sys.size());
        else
            hipLaunchKernelGGL((kz_fast_batch<T, NZ, L, false>), grid, dim3(kThreads), 0, s, tab, blks,
                               (int)g.sys.size());
    }
}

template <typename T, int NZ>
void launch_kz_batch_n(lise_batch* b, const BatchGroup& g, int st, int ph, bool nt, hipStream_t s) {
    if (g.zl == 4) launch_kz_batch_l<T, NZ, 4>(b, g, st, ph, nt, s);
    else if (g.zl == 2) launch_kz_batch_l<T, NZ, 2>(b, g, st, ph, nt, s);
    else launch_kz_batch_l<T, NZ, 1>(b, g, st, ph, nt, s);
}

template <typename T>
int launch_kz_batch(lise_batch* b, const BatchGroup& g, int st, int ph, hipStream_t s) {
    const bool nt = b->sys[g.sys[0]]->stream_hint;
    hipEvent_t ev;
    bprof_begin(b, &ev, s);
    switch (g.nz) {
        case 8: launch_kz_batch_n<T, 8>(b, g, st, ph, nt, s); break;
        case 16: launch_kz_batch_n<T, 16>(b, g, st, ph, nt, s); break;
        case 20: launch_kz_batch_n<T, 20>(b, g, st, ph, nt, s); break;
        case 24: launch_kz_batch_n<T, 24>(b, g, st, ph, nt, s); break;
        case 32: launch_kz_batch_n<T, 32>(b, g, st, ph, nt, s); break;
        case 48: launch_kz_batch_n<T, 48>(b, g, st, ph, nt, s); break;
        default: launch_kz_batch_n<T, 64>(b, g, st, ph, nt, s); break;
    }
    bprof_end(b, 1, ev, s);
    return bcheck_launch(b, "kz_fast_batch");
}

template <typename T>
int batch_phase_group(lise_batch* b, const BatchGroup& g, int st, int ph, hipStream_t s) {
    if (!g.cube) BCHK(launch_kz_batch<T>(b, g, st, ph, s));
    const int rc = ph == 0 ? launch_kp_batch<T, KP_ABM1>(b, g, st, s) : launch_kp_batch<T, KP_ABM2>(b, g, st, s);
    if (rc != LISE_OK) return rc;
    if (!g.dens_split) return LISE_OK;
    const char* base = static_cast<const char*>(b->dtab);
    hipEvent_t ev;
    bprof_begin(b, &ev, s);
    hipLaunchKernelGGL((dens_batch_kernel<T>), dim3((unsigned)g.dblocks), dim3(kThreads), 0, s,
                       reinterpret_cast<const DensDesc<T>*>(base + g.off_dens[st][ph]),
                       reinterpret_cast<const long long*>(base + g.off_dblks), (int)g.sys.size());
    bprof_end(b, 2, ev, s);
    return bcheck_launch(b, "dens_batch_kernel");
}

// One ABM step of every grouped system (the enqueue only): per phase, the
// z-axis and plane launches of each group, then one density + fields launch
// for all systems; last, every system's time advances by dt.  `st` is the
// step's place in the ring period relative to the tables' base state.
int batch_step_grouped(lise_batch* b, int st, hipStream_t s) {
    const char* base = static_cast<const char*>(b->dtab);
    for (int ph = 0; ph < 2; ++ph) {
        for (const auto& g : b->groups) {
            if (g.prec == LISE_FP64) BCHK(batch_phase_group<double>(b, g, st, ph, s));
            else BCHK(batch_phase_group<float>(b, g, st, ph, s));
        }
        hipEvent_t ev;
        bprof_begin(b, &ev, s);
        hipLaunchKernelGGL(fields_batch_kernel, dim3((unsigned)b->fblocks), dim3(kFieldPts * kFieldGroups), 0, s,
                           reinterpret_cast<const FieldsDesc*>(base + b->off_fd[ph]),
                           reinterpret_cast<const long long*>(base + b->off_fblks), (int)b->grouped.size(), b->tab_dt);
        bprof_end(b, 2, ev, s);
        BCHK(bcheck_launch(b, "fields_batch_kernel"));
    }
    const int n = (int)b->grouped.size();
    hipLaunchKernelGGL(tick_batch_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s,
                       reinterpret_cast<double* const*>(base + b->off_tick), n, b->tab_dt);
    return bcheck_launch(b, "tick_batch_kernel");
}

void batch_advance_host(lise_batch* b) {
    for (int i : b->grouped) advance_host(b->sys[i], b->tab_dt);
    b->tphase = (b->tphase + 1) % kBatchPeriod;
}

// Capture one ring period of grouped steps (starting at tphase 0) on the
// internal stream: kernel nodes only, no events or forks inside the capture.
int batch_capture(lise_batch* b) {
    if (b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
    }
    hipError_t e = hipEventRecord(b->ev_cap, b->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->cap, b->ev_cap, 0);
    if (e == hipSuccess) e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bfail(b, LISE_E_HIP, "begin capture: %s", hipGetErrorString(e));
    const bool prof = b->prof.on;
    b->prof.on = false;
    int rc = LISE_OK;
    for (int st = 0; st < kBatchPeriod && rc == LISE_OK; ++st) rc = batch_step_grouped(b, st, b->cap);
    b->prof.on = prof;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->cap, &g);
    if (rc != LISE_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        if (rc != LISE_OK) return rc;
        return bfail(b, LISE_E_HIP, "end capture: %s", hipGetErrorString(e));
    }
    e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->gexec = nullptr;
        return bfail(b, LISE_E_HIP, "graph instantiation: %s", hipGetErrorString(e));
    }
    return LISE_OK;
}

// ---- checkpoint files ----------------------------------------------------------------
// Layout (little-endian): CkptHeader, then arrays of M*C*N complex numbers in
// the context's own precision: y_n; with history also y_{n-1}, y'_{n-1},
// y'_{n-2}, y'_{n-3}, p_n - c_n and the densities (3N float64: n, Re kappa,
// Im kappa) of y_n; last the reference norms (M float64).

struct CkptHeader {
    char magic[8];
    int32_t version, ncomp, precision, nx, ny, nz, history, elem_bytes;
    double a;
    int64_t M;
    double t;
    int64_t step;
    double dt;
    int64_t reserved[4];
};
static_assert(sizeof(CkptHeader) == 112, "checkpoint header layout");
constexpr char kCkptMagic[8] = {'L', 'I', 'S', 'E', 'C', 'K', 'P', '1'};

// Pinned staging, two buffers so that one copy engine transfer overlaps the
// file I/O of the other buffer.
struct Staging {
    void* h[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    size_t cap = 0;
    ~Staging() {
        for (int i = 0; i < 2; ++i) {
            if (ev[i]) (void)hipEventSynchronize(ev[i]), (void)hipEventDestroy(ev[i]);
            if (h[i]) (void)hipHostFree(h[i]);
        }
    }
};

int staging_init(lise_ctx* c, Staging* st, size_t cap) {
    st->cap = cap;
    for (int i = 0; i < 2; ++i) {
        HIPCHK(c, hipHostMalloc(&st->h[i], cap, hipHostMallocDefault));
        HIPCHK(c, hipEventCreateWithFlags(&st->ev[i], hipEventDisableTiming));
    }
    return LISE_OK;
}

// device -> file, in pieces of the staging size
int write_device(lise_ctx* c, Staging* st, FILE* f, const void* dev, size_t bytes) {
    const char* src = static_cast<const char*>(dev);
    const size_t np = (bytes + st->cap - 1) / st->cap;
    if (np == 0) return LISE_OK;
    HIPCHK(c, hipMemcpyAsync(st->h[0], src, std::min(st->cap, bytes), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipEventRecord(st->ev[0], c->stream));
    for (size_t i = 0; i < np; ++i) {
        const int b = (int)(i & 1);
        const size_t off = i * st->cap, len = std::min(st->cap, bytes - off);
        if (i + 1 < np) {
            const size_t o2 = off + st->cap, l2 = std::min(st->cap, bytes - o2);
            HIPCHK(c, hipMemcpyAsync(st->h[1 - b], src + o2, l2, hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipEventRecord(st->ev[1 - b], c->stream));
        }
        HIPCHK(c, hipEventSynchronize(st->ev[b]));
        if (fwrite(st->h[b], 1, len, f) != len) return fail(c, LISE_E_ARG, "checkpoint write failed");
        // the next copy into this buffer is issued only after the write above
    }
    return LISE_OK;
}

// file -> device, in pieces of the staging size
int read_device(lise_ctx* c, Staging* st, FILE* f, void* dev, size_t bytes) {
    char* dst = static_cast<char*>(dev);
    for (size_t off = 0, i = 0; off < bytes; off += st->cap, ++i) {
        const int b = (int)(i & 1);
        const size_t len = std::min(st->cap, bytes - off);
        HIPCHK(c, hipEventSynchronize(st->ev[b]));   // the previous copy out of this buffer is done
        if (fread(st->h[b], 1, len, f) != len) return fail(c, LISE_E_ARG, "checkpoint file truncated");
        HIPCHK(c, hipMemcpyAsync(dst + off, st->h[b], len, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipEventRecord(st->ev[b], c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LISE_OK;
}

}  // namespace


// =============================================================================
// C-ABI

extern "C" {

int lise_init(lise_ctx** out, const lise_lattice* lat, int64_t n_qpwf, const lise_functional* fn, void* hip_stream) {
    if (!out || !lat || !fn) return LISE_E_ARG;
    *out = nullptr;
    lise_ctx* c = new (std::nothrow) lise_ctx();
    if (!c) return LISE_E_NOMEM;
    auto bail = [&](int rc) {
        fprintf(stderr, "lise_init: %s\n", c->err);
        lise_free(c);
        return rc;
    };
    c->lat = *lat;
    c->fn = *fn;
    if (!(lat->a > 0.0)) return bail(fail(c, LISE_E_ARG, "lattice spacing must be positive"));
    if (!valid_dim(lat->nx) || !valid_dim(lat->ny) || !valid_dim(lat->nz))
        return bail(fail(c, LISE_E_UNSUPPORTED, "lattice %dx%dx%d: each side must be 1..128 with prime factors 2,3,5",
                         lat->nx, lat->ny, lat->nz));
    if (n_qpwf < 1) return bail(fail(c, LISE_E_ARG, "n_qpwf must be >= 1"));
    if (fn->ncomp != 2 && fn->ncomp != 4) return bail(fail(c, LISE_E_ARG, "ncomp must be 2 or 4"));
    if (fn->regularize != 0 && fn->regularize != 1) return bail(fail(c, LISE_E_ARG, "regularize must be 0 or 1"));
    if (fn->remove_phase != 0 && fn->remove_phase != 1) return bail(fail(c, LISE_E_ARG, "remove_phase must be 0 or 1"));
    c->remove_phase = fn->remove_phase;
    if (fn->reserved != 0) return bail(fail(c, LISE_E_ARG, "lise_functional.reserved must be 0"));
    if (!lise::plan::effective_coupling(fn->g, lat->a, fn->regularize, &c->g_used))
        return bail(fail(c, LISE_E_ARG, "regularised coupling undefined (g = 0 or 1/g = K / (4 pi a))"));
    if (fn->precision != LISE_FP64 && fn->precision != LISE_FP32 && fn->precision != LISE_FP32_MFMA)
        return bail(fail(c, LISE_E_UNSUPPORTED, "precision %d not supported", fn->precision));
    if (fn->precision == LISE_FP32_MFMA && !(lat->nx == lat->ny && mfma_side(lat->nx)))
        return bail(fail(c, LISE_E_UNSUPPORTED, "the MFMA form needs square xy-planes of side 16, 32, 48 or 64"));
    c->C = fn->ncomp;
    c->mfma_mode = fn->precision == LISE_FP32_MFMA ? 1 : 0;
    c->prec = fn->precision == LISE_FP64 ? LISE_FP64 : LISE_FP32;
    c->esz = c->prec == LISE_FP64 ? 16 : 8;
    c->M = n_qpwf;
    try {
        c->set_mask.assign((size_t)n_qpwf, 0);
    } catch (...) {
        return bail(fail(c, LISE_E_NOMEM, "host allocation of the qpwf coverage map failed"));
    }
    c->N = (long long)lat->nx * lat->ny * lat->nz;
    c->per = (long long)c->C * c->N;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    hipError_t e = hipGetDevice(&c->device);
    if (e != hipSuccess) return bail(fail(c, LISE_E_HIP, "hipGetDevice: %s", hipGetErrorString(e)));
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, c->device);
    if (e != hipSuccess) return bail(fail(c, LISE_E_HIP, "hipGetDeviceProperties: %s", hipGetErrorString(e)));
    c->lds_limit = prop.sharedMemPerBlock;
    set_all_attrs((int)c->lds_limit);
    {
        // the device's own address of the fixed staging array, once per device
        if (c->device < 0 || c->device >= kMaxDevices)
            return bail(fail(c, LISE_E_UNSUPPORTED, "device index %d beyond %d", c->device, kMaxDevices));
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_addr[c->device]) {
            void* p = nullptr;
            e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return bail(fail(c, LISE_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e)));
            g_scratch_addr[c->device] = p;
        }
        c->scratch_dev = g_scratch_addr[c->device];
    }
    // plans and twiddles
    std::vector<cpx<double>> tw;
    if (!make_plan(lat->nx, &c->px, &tw) || !make_plan(lat->ny, &c->py, &tw) || !make_plan(lat->nz, &c->pz, &tw))
        return bail(fail(c, LISE_E_UNSUPPORTED, "no FFT plan"));
    // W_n^j tables (j < n) for the register-FFT kernels
    auto full_table = [&](int n) { return plan::full_table(n, &tw); };
    if (lat->nx == lat->ny && fast_side(lat->nx)) c->tw_full_xy = full_table(lat->nx);
    if (fast_side(lat->nz)) c->tw_full_z = full_table(lat->nz);
    if (c->prec == LISE_FP64) {
        int rc = dalloc(c, &c->tw, tw.size() * sizeof(cpx<double>));
        if (rc) return bail(rc);
        e = hipMemcpy(c->tw, tw.data(), tw.size() * sizeof(cpx<double>), hipMemcpyHostToDevice);
    } else {
        std::vector<cpx<float>> tf(tw.size());
        for (size_t i = 0; i < tw.size(); ++i) {
            tf[i].re = (float)tw[i].re;
            tf[i].im = (float)tw[i].im;
        }
        int rc = dalloc(c, &c->tw, tf.size() * sizeof(cpx<float>));
        if (rc) return bail(rc);
        e = hipMemcpy(c->tw, tf.data(), tf.size() * sizeof(cpx<float>), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return bail(fail(c, LISE_E_HIP, "twiddle upload: %s", hipGetErrorString(e)));
    if (c->mfma_mode) {
        const std::vector<unsigned short> dk = kinetic_matrix_bf16(lat->nx, lat->a);
        int rc0 = dalloc(c, reinterpret_cast<void**>(&c->dkin), dk.size() * sizeof(short));
        if (rc0) return bail(rc0);
        e = hipMemcpy(c->dkin, dk.data(), dk.size() * sizeof(short), hipMemcpyHostToDevice);
        if (e != hipSuccess) return bail(fail(c, LISE_E_HIP, "kinetic table upload: %s", hipGetErrorString(e)));
    }
    const size_t state_bytes = (size_t)c->M * c->per * c->esz;
    for (int i = 0; i < 7; ++i) {
        int rc = dalloc(c, &c->buf[i], state_bytes);
        if (rc) return bail(rc);
    }
    const size_t nb = (size_t)c->N * sizeof(double);
    int rc = LISE_OK;
    rc = rc ? rc : dalloc(c, reinterpret_cast<void**>(&c->dens_cur), 3 * nb);
    rc = rc ? rc : dalloc(c, reinterpret_cast<void**>(&c->dens_tmp), 3 * nb);
    rc = rc ? rc : dalloc(c, reinterpret_cast<void**>(&c->V_cur), nb);
    rc = rc ? rc : dalloc(c, reinterpret_cast<void**>(&c->V_tmp), nb);
    rc = rc ? rc : dalloc(c, reinterpret_cast<void**>(&c->D_cur), 2 * nb);
    rc = rc ? rc : dalloc(c, reinterpret_cast<void**>(&c->D_tmp), 2 * nb);
    rc = rc ? rc : dalloc(c, reinterpret_cast<void**>(&c->norms), (size_t)c->M * sizeof(double));
    rc = rc ? rc : dalloc(c, reinterpret_cast<void**>(&c->norms0), (size_t)c->M * sizeof(double));
    rc = rc ? rc : dalloc(c, reinterpret_cast<void**>(&c->bad), sizeof(int));
    rc = rc ? rc : dalloc(c, reinterpret_cast<void**>(&c->dtime), sizeof(double));
    if (rc) return bail(rc);
    e = hipMemset(c->dtime, 0, sizeof(double));
    if (e == hipSuccess) e = hipMemset(c->bad, 0, sizeof(int));
    if (e != hipSuccess) return bail(fail(c, LISE_E_HIP, "hipMemset: %s", hipGetErrorString(e)));
    e = hipStreamCreateWithFlags(&c->s2, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_cap, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_start, hipEventDisableTiming);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
        e = hipEventCreateWithFlags(&c->ev_kz[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_kp[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) return bail(fail(c, LISE_E_HIP, "stream/event creation: %s", hipGetErrorString(e)));
    rc = configure(c);
    if (rc) return bail(rc);
    *out = c;
    return LISE_OK;
}

int lise_set_qpwf(lise_ctx* c, int64_t first, int64_t count, const void* src, int32_t src_is_device) {
    if (!c || !src) return LISE_E_ARG;
    if (first < 0 || count < 1 || first + count > c->M) return fail(c, LISE_E_ARG, "qpwf range out of bounds");
    const long long n = count * c->per;
    void* dst = static_cast<char*>(c->buf[0]) + (size_t)first * c->per * c->esz;
    if (c->hist || c->iy != 0) {
        // a previous evolution moved y_n away from buffer 0 (or left history
        // behind it): start over there, and require the whole set again
        c->iy = 0;
        reset_coverage(c);
    }
    if (c->prec == LISE_FP64) {
        HIPCHK(c, hipMemcpyAsync(dst, src, (size_t)n * 16, src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                 c->stream));
    } else {
        // stage float64 through device memory (p - c slot has room for M qpwfs in fp32: convert in pieces)
        const long long piece = std::max<long long>(1, (64LL << 20) / 16);
        void* stage = nullptr;
        CHK(dalloc(c, &stage, (size_t)std::min<long long>(piece, n) * 16));
        for (long long o = 0; o < n; o += piece) {
            const long long k = std::min<long long>(piece, n - o);
            const char* s = static_cast<const char*>(src) + (size_t)o * 16;
            hipError_t e = hipMemcpyAsync(stage, s, (size_t)k * 16,
                                          src_is_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream);
            if (e != hipSuccess) {
                (void)hipStreamSynchronize(c->stream);
                dfree(&stage);
                return fail(c, LISE_E_HIP, "qpwf upload: %s", hipGetErrorString(e));
            }
            hipLaunchKernelGGL((convert_kernel<float, double>), dim3(2048), dim3(kThreads), 0, c->stream,
                               reinterpret_cast<const cpx<double>*>(stage),
                               reinterpret_cast<cpx<float>*>(dst) + o, k);
        }
        (void)hipStreamSynchronize(c->stream);
        dfree(&stage);
        CHK(check_launch(c, "convert_kernel"));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (long long j = first; j < first + count; ++j)
        if (!c->set_mask[j]) {
            c->set_mask[j] = 1;
            ++c->n_set;
        }
    c->hist = false;
    c->dens_valid = false;
    if (c->n_set >= c->M) {
        if (c->prec == LISE_FP64) CHK(norms_t<double>(c, c->norms0));
        else CHK(norms_t<float>(c, c->norms0));
        c->norms0_valid = true;
    }
    return LISE_OK;
}

int lise_get_qpwf(lise_ctx* c, int64_t first, int64_t count, void* dst, int32_t dst_is_device) {
    if (!c || !dst) return LISE_E_ARG;
    if (first < 0 || count < 1 || first + count > c->M) return fail(c, LISE_E_ARG, "qpwf range out of bounds");
    const long long n = count * c->per;
    const char* src = static_cast<const char*>(c->buf[c->iy]) + (size_t)first * c->per * c->esz;
    if (c->prec == LISE_FP64) {
        HIPCHK(c, hipMemcpyAsync(dst, src, (size_t)n * 16, dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                 c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return LISE_OK;
    }
    const long long piece = (64LL << 20) / 16;
    void* stage = nullptr;
    CHK(dalloc(c, &stage, (size_t)std::min<long long>(piece, n) * 16));
    int rc = LISE_OK;
    for (long long o = 0; o < n && rc == LISE_OK; o += piece) {
        const long long k = std::min<long long>(piece, n - o);
        hipLaunchKernelGGL((convert_kernel<double, float>), dim3(2048), dim3(kThreads), 0, c->stream,
                           reinterpret_cast<const cpx<float>*>(src) + o, reinterpret_cast<cpx<double>*>(stage), k);
        hipError_t e = hipMemcpyAsync(static_cast<char*>(dst) + (size_t)o * 16, stage, (size_t)k * 16,
                                      dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) rc = fail(c, LISE_E_HIP, "qpwf download: %s", hipGetErrorString(e));
    }
    (void)hipStreamSynchronize(c->stream);
    dfree(&stage);
    return rc;
}

int lise_apply_h(lise_ctx* c, int64_t first, int64_t count, void* out, int32_t out_is_device) {
    if (!c || !out) return LISE_E_ARG;
    if (first < 0 || count < 1 || first + count > c->M) return fail(c, LISE_E_ARG, "qpwf range out of bounds");
    return c->prec == LISE_FP64 ? apply_h_t<double>(c, first, count, out, out_is_device)
                                : apply_h_t<float>(c, first, count, out, out_is_device);
}

int lise_apply_h_noalloc(lise_ctx* c, int64_t first, int64_t count, void* out_device) {
    if (!c || !out_device) return LISE_E_ARG;
    if (first < 0 || count < 1 || first + count > c->M) return fail(c, LISE_E_ARG, "qpwf range out of bounds");
    return c->prec == LISE_FP64 ? apply_h_noalloc_t<double>(c, first, count, out_device)
                                : apply_h_noalloc_t<float>(c, first, count, out_device);
}

int lise_startup(lise_ctx* c, double dt) {
    if (!c) return LISE_E_ARG;
    if (!(std::isfinite(dt)) || dt == 0.0) return fail(c, LISE_E_ARG, "dt must be finite and non-zero");
    return c->prec == LISE_FP64 ? startup_t<double>(c, dt) : startup_t<float>(c, dt);
}

int lise_step(lise_ctx* c, double dt, int64_t nsteps) {
    if (!c) return LISE_E_ARG;
    if (!(std::isfinite(dt)) || dt == 0.0) return fail(c, LISE_E_ARG, "dt must be finite and non-zero");
    if (nsteps < 0) return fail(c, LISE_E_ARG, "nsteps must be >= 0");
    if (c->n_set < c->M) return fail(c, LISE_E_STATE, "qpwfs not fully set");
    return c->prec == LISE_FP64 ? step_t<double>(c, dt, nsteps) : step_t<float>(c, dt, nsteps);
}

int lise_densities(lise_ctx* c, double* n_out, double* kappa_out, int32_t out_is_device) {
    if (!c) return LISE_E_ARG;
    CHK(c->prec == LISE_FP64 ? ensure_fields_t<double>(c) : ensure_fields_t<float>(c));
    const size_t nb = (size_t)c->N * sizeof(double);
    const hipMemcpyKind kind = out_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (n_out) HIPCHK(c, hipMemcpyAsync(n_out, c->dens_cur, nb, kind, c->stream));
    if (kappa_out) {
        // kappa is stored as two real planes; interleave through a small staging copy
        std::vector<double> re(c->N), im(c->N);
        HIPCHK(c, hipMemcpyAsync(re.data(), c->dens_cur + c->N, nb, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(im.data(), c->dens_cur + 2 * c->N, nb, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        std::vector<double> il(2 * c->N);
        for (long long r = 0; r < c->N; ++r) {
            il[2 * r] = re[r];
            il[2 * r + 1] = im[r];
        }
        HIPCHK(c, hipMemcpyAsync(kappa_out, il.data(), 2 * nb, out_is_device ? hipMemcpyHostToDevice : hipMemcpyHostToHost,
                                 c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LISE_OK;
}

int lise_observables(lise_ctx* c, lise_obs* out) {
    if (!c || !out) return LISE_E_ARG;
    return c->prec == LISE_FP64 ? observables_t<double>(c, out) : observables_t<float>(c, out);
}

int lise_get_time(const lise_ctx* c, double* t, int64_t* step) {
    if (!c) return LISE_E_ARG;
    if (t) *t = c->t;
    if (step) *step = c->step;
    return LISE_OK;
}

int lise_set_time(lise_ctx* c, double t) {
    if (!c || !std::isfinite(t)) return LISE_E_ARG;
    HIPCHK(c, hipMemcpyAsync(c->dtime, &t, sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->t = t;
    c->hist = false;
    return LISE_OK;
}

int lise_set_stream(lise_ctx* c, void* hip_stream) {
    if (!c) return LISE_E_ARG;
    c->stream = reinterpret_cast<hipStream_t>(hip_stream);
    return LISE_OK;
}

int lise_set_tuning(lise_ctx* c, const lise_tuning* t) {
    if (!c || !t) return LISE_E_ARG;
    if (t->chunk_qpwf < 0 || t->jgroup < 0) return fail(c, LISE_E_ARG, "negative tuning value");
    if (t->z_lanes != 0 && t->z_lanes != 1 && t->z_lanes != 2 && t->z_lanes != 4)
        return fail(c, LISE_E_ARG, "z_lanes must be 0, 1, 2 or 4");
    if (t->z_dense < -1 || t->z_dense > 1) return fail(c, LISE_E_ARG, "z_dense must be -1, 0 or 1");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->s2) HIPCHK(c, hipStreamSynchronize(c->s2));
    c->chunk = t->chunk_qpwf;
    c->jg_user = t->jgroup;
    c->single_pass = t->single_pass < 0 ? -1 : (t->single_pass > 0 ? 1 : 0);
    c->zl_user = t->z_lanes;
    c->z_dense_user = t->z_dense;
    c->fused_mode = t->fused < 0 ? -1 : (t->fused > 0 ? 1 : 0);
    c->generic = t->generic ? 1 : 0;
    c->overlap = t->no_overlap ? 0 : 1;
    c->use_graph = t->graph ? 1 : 0;
    return configure(c);
}

int lise_profile(lise_ctx* c, int32_t enable) {
    if (!c) return LISE_E_ARG;
    if (enable && c->prof.pool.empty()) {
        c->prof.pool.resize(1 << 14);
        for (auto& ev : c->prof.pool) HIPCHK(c, hipEventCreate(&ev));
    }
    c->prof.on = enable != 0;
    return LISE_OK;
}

int lise_profile_read(lise_ctx* c, int32_t which, int64_t* launches, double* total_ms) {
    if (!c || which < 0 || which > 4) return LISE_E_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto& r : c->prof.recs) {
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, r.a, r.b));
        c->prof.total_ms[r.cls] += ms;
        c->prof.count[r.cls] += 1;
    }
    c->prof.recs.clear();
    c->prof.used = 0;
    if (launches) *launches = c->prof.count[which];
    if (total_ms) *total_ms = c->prof.total_ms[which];
    c->prof.total_ms[which] = 0.0;
    c->prof.count[which] = 0;
    if (c->prof.overflow) {
        c->prof.overflow = false;
        return fail(c, LISE_E_STATE, "profiling event pool exhausted: read the counters more often");
    }
    return LISE_OK;
}

int lise_memory(const lise_ctx* c, int64_t* bytes) {
    if (!c || !bytes) return LISE_E_ARG;
    long long b = 7LL * c->M * c->per * (long long)c->esz;
    b += (c->Gbuf[1] ? 2 : 1) * c->g_cap * c->per * (long long)c->esz;
    b += (long long)c->slot_cap * 3 * c->N * 8;
    b += 10LL * c->N * 8;
    b += (long long)c->ah_cap;
    *bytes = b;
    return LISE_OK;
}

int lise_save(lise_ctx* c, const char* path, int32_t with_history) {
    if (!c || !path) return LISE_E_ARG;
    if (with_history != 0 && with_history != 1) return fail(c, LISE_E_ARG, "with_history must be 0 or 1");
    if (c->n_set < c->M) return fail(c, LISE_E_STATE, "qpwfs not fully set");
    if (with_history && !c->hist) return fail(c, LISE_E_STATE, "no ABM history to save (step first)");
    CkptHeader h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, kCkptMagic, 8);
    h.version = 1;
    h.ncomp = c->C;
    h.precision = c->fn.precision;
    h.nx = c->lat.nx;
    h.ny = c->lat.ny;
    h.nz = c->lat.nz;
    h.history = with_history;
    h.elem_bytes = (int32_t)c->esz;
    h.a = c->lat.a;
    h.M = c->M;
    h.t = c->t;
    h.step = c->step;
    h.dt = with_history ? c->dt_hist : 0.0;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    FILE* f = fopen(path, "wb");
    if (!f) return fail(c, LISE_E_ARG, "cannot open %s for writing", path);
    Staging st;
    int rc = staging_init(c, &st, 64u << 20);
    if (rc == LISE_OK && fwrite(&h, sizeof(h), 1, f) != 1) rc = fail(c, LISE_E_ARG, "checkpoint write failed");
    const size_t arr = (size_t)c->M * c->per * c->esz;
    std::vector<int> bufs = {c->iy};
    if (with_history) {
        bufs.push_back(1 - c->iy);
        for (int k = 3; k >= 1; --k) bufs.push_back(2 + (c->dn + k) % 4);   // y'_{n-1}, y'_{n-2}, y'_{n-3}
        bufs.push_back(6);
    }
    for (int b : bufs)
        if (rc == LISE_OK) rc = write_device(c, &st, f, c->buf[b], arr);
    if (rc == LISE_OK && with_history) rc = write_device(c, &st, f, c->dens_cur, 3 * (size_t)c->N * sizeof(double));
    if (rc == LISE_OK) rc = write_device(c, &st, f, c->norms0, (size_t)c->M * sizeof(double));
    if (fclose(f) != 0 && rc == LISE_OK) rc = fail(c, LISE_E_ARG, "checkpoint close failed");
    return rc;
}

int lise_load(lise_ctx* c, const char* path) {
    if (!c || !path) return LISE_E_ARG;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    FILE* f = fopen(path, "rb");
    if (!f) return fail(c, LISE_E_ARG, "cannot open %s", path);
    CkptHeader h;
    int rc = LISE_OK;
    if (fread(&h, sizeof(h), 1, f) != 1 || std::memcmp(h.magic, kCkptMagic, 8) != 0 || h.version != 1)
        rc = fail(c, LISE_E_ARG, "%s is not a version-1 checkpoint", path);
    else if (h.ncomp != c->C || h.precision != c->fn.precision || h.nx != c->lat.nx || h.ny != c->lat.ny ||
             h.nz != c->lat.nz || h.a != c->lat.a || h.M != c->M || h.elem_bytes != (int32_t)c->esz ||
             (h.history != 0 && h.history != 1))
        rc = fail(c, LISE_E_ARG, "checkpoint does not match the context (lattice, C, M or precision)");
    else if (!std::isfinite(h.t) || (h.history && !(std::isfinite(h.dt) && h.dt != 0.0)))
        rc = fail(c, LISE_E_ARG, "checkpoint holds a non-finite time or step size");
    Staging st;
    if (rc == LISE_OK) rc = staging_init(c, &st, 64u << 20);
    const size_t arr = (size_t)c->M * c->per * c->esz;
    // canonical placement: y_n in buffer 0, y_{n-1} in 1, derivatives as after dn = 0
    std::vector<int> bufs = {0};
    if (h.history && rc == LISE_OK) {
        bufs.push_back(1);
        for (int k = 3; k >= 1; --k) bufs.push_back(2 + k % 4);
        bufs.push_back(6);
    }
    for (int b : bufs)
        if (rc == LISE_OK) rc = read_device(c, &st, f, c->buf[b], arr);
    if (rc == LISE_OK && h.history) rc = read_device(c, &st, f, c->dens_cur, 3 * (size_t)c->N * sizeof(double));
    if (rc == LISE_OK) rc = read_device(c, &st, f, c->norms0, (size_t)c->M * sizeof(double));
    fclose(f);
    if (rc != LISE_OK) {
        // the state may be partly overwritten: require a fresh set
        reset_coverage(c);
        c->hist = false;
        c->dens_valid = false;
        return rc;
    }
    c->iy = 0;
    c->dn = 0;
    std::fill(c->set_mask.begin(), c->set_mask.end(), (unsigned char)1);
    c->n_set = c->M;
    c->norms0_valid = true;
    c->t = h.t;
    c->step = h.step;
    c->config_version += 1;    // buffer roles changed: no stale graph replays
    HIPCHK(c, hipMemcpyAsync(c->dtime, &c->t, sizeof(double), hipMemcpyHostToDevice, c->stream));
    if (h.history) {
        c->hist = true;
        c->dt_hist = h.dt;
        c->dens_valid = true;
        CHK(launch_fields(c, 0, nullptr, c->dens_cur, c->V_cur, c->D_cur, 0.0));
    } else {
        c->hist = false;
        c->dens_valid = false;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LISE_OK;
}

int lise_batch_create(lise_batch** out, int32_t nsys, lise_ctx* const* ctxs, void* hip_stream) {
    if (!out || nsys < 1 || !ctxs) return LISE_E_ARG;
    *out = nullptr;
    lise_batch* b = new (std::nothrow) lise_batch();
    if (!b) return LISE_E_NOMEM;
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    for (int i = 0; i < nsys; ++i) {
        if (!ctxs[i]) {
            delete b;
            return LISE_E_ARG;
        }
        for (int k = 0; k < i; ++k)
            if (ctxs[k] == ctxs[i]) {
                delete b;
                return LISE_E_ARG;
            }
        b->sys.push_back(ctxs[i]);
    }
    hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_cap, hipEventDisableTiming);
    if (e != hipSuccess) {
        lise_batch_free(b);
        return LISE_E_HIP;
    }
    // earlier work of every system completes before the batch takes it over
    for (lise_ctx* c : b->sys) {
        (void)hipStreamSynchronize(c->stream);
        c->stream = b->stream;
    }
    *out = b;
    return LISE_OK;
}

int lise_batch_set_graph(lise_batch* b, int32_t enable) {
    if (!b || (enable != 0 && enable != 1)) return LISE_E_ARG;
    b->use_graph = enable;
    return LISE_OK;
}

int lise_batch_step(lise_batch* b, double dt, int64_t nsteps) {
    if (!b) return LISE_E_ARG;
    if (!std::isfinite(dt) || dt == 0.0 || nsteps < 0) return bfail(b, LISE_E_ARG, "bad dt or nsteps");
    for (size_t i = 0; i < b->sys.size(); ++i) {
        lise_ctx* c = b->sys[i];
        c->stream = b->stream;
        if (c->n_set < c->M) return bfail(b, LISE_E_STATE, "system %zu: qpwfs not fully set", i);
    }
    // start-up where a system has no history for this dt (one system at a time)
    for (size_t i = 0; i < b->sys.size(); ++i) {
        lise_ctx* c = b->sys[i];
        if (c->hist && c->dt_hist == dt) continue;
        int rc = c->prec == LISE_FP64 ? startup_t<double>(c, dt) : startup_t<float>(c, dt);
        if (rc != LISE_OK) return bfail(b, rc, "system %zu start-up: %s", i, c->err);
        if (c->gexec) {
            (void)hipGraphExecDestroy(c->gexec);
            c->gexec = nullptr;
        }
    }
    if (!batch_tables_valid(b, dt)) BCHK(batch_build(b, dt));
    if (!b->grouped.empty()) {
        long long left = nsteps;
        // eager steps up to the start of a ring period, then graph replays
        while (left > 0 && (b->tphase != 0 || !b->use_graph || b->prof.on || left < kBatchPeriod)) {
            BCHK(batch_step_grouped(b, b->tphase, b->stream));
            batch_advance_host(b);
            --left;
        }
        if (left >= kBatchPeriod) {
            if (!b->gexec) BCHK(batch_capture(b));
            for (; left >= kBatchPeriod; left -= kBatchPeriod) {
                hipError_t e = hipGraphLaunch(b->gexec, b->stream);
                if (e != hipSuccess) return bfail(b, LISE_E_HIP, "graph launch: %s", hipGetErrorString(e));
                for (int k = 0; k < kBatchPeriod; ++k) batch_advance_host(b);
            }
        }
        for (; left > 0; --left) {
            BCHK(batch_step_grouped(b, b->tphase, b->stream));
            batch_advance_host(b);
        }
    }
    for (int i : b->solo) {
        lise_ctx* c = b->sys[i];
        int rc = advance_any(c, dt, nsteps);
        if (rc != LISE_OK) return bfail(b, rc, "system %d: %s", i, c->err);
    }
    for (size_t k = 0; k < b->sys.size(); ++k) {
        int rc = check_bad(b->sys[k]);
        if (rc != LISE_OK) return bfail(b, rc, "system %zu: %s", k, b->sys[k]->err);
    }
    return LISE_OK;
}

int lise_batch_info(const lise_batch* b, int32_t* ngroups, int32_t* nsolo) {
    if (!b) return LISE_E_ARG;
    if (ngroups) *ngroups = (int32_t)b->groups.size();
    if (nsolo) *nsolo = (int32_t)b->solo.size();
    return LISE_OK;
}

int lise_batch_profile(lise_batch* b, int32_t enable) {
    if (!b) return LISE_E_ARG;
    if (enable && b->prof.pool.empty()) {
        b->prof.pool.resize(1 << 14);
        for (auto& ev : b->prof.pool)
            if (hipEventCreate(&ev) != hipSuccess) return bfail(b, LISE_E_HIP, "event pool");
    }
    b->prof.on = enable != 0;
    return LISE_OK;
}

int lise_batch_profile_read(lise_batch* b, int32_t which, int64_t* launches, double* total_ms) {
    if (!b || which < 0 || which > 3) return LISE_E_ARG;
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, LISE_E_HIP, "%s", hipGetErrorString(e));
    for (auto& r : b->prof.recs) {
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) return bfail(b, LISE_E_HIP, "%s", hipGetErrorString(e));
        b->prof.total_ms[r.cls] += ms;
        b->prof.count[r.cls] += 1;
    }
    b->prof.recs.clear();
    b->prof.used = 0;
    if (launches) *launches = b->prof.count[which];
    if (total_ms) *total_ms = b->prof.total_ms[which];
    b->prof.total_ms[which] = 0.0;
    b->prof.count[which] = 0;
    if (b->prof.overflow) {
        b->prof.overflow = false;
        return bfail(b, LISE_E_STATE, "profiling event pool exhausted: read the counters more often");
    }
    return LISE_OK;
}

const char* lise_batch_last_error(const lise_batch* b) { return b ? b->err : "null batch"; }

void lise_batch_free(lise_batch* b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    else (void)hipDeviceSynchronize();
    if (b->cap) (void)hipStreamSynchronize(b->cap);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->ev_cap) (void)hipEventDestroy(b->ev_cap);
    for (auto& ev : b->prof.pool) (void)hipEventDestroy(ev);
    dfree(&b->G);
    dfree(&b->dtab);
    delete b;
}

int lise_autotune(lise_ctx* c, double dt, int32_t trial_steps, lise_tuning* chosen) {
    if (!c || trial_steps < 1) return LISE_E_ARG;
    if (!std::isfinite(dt) || dt == 0.0) return fail(c, LISE_E_ARG, "dt must be finite and non-zero");
    if (c->n_set < c->M) return fail(c, LISE_E_STATE, "qpwfs not fully set");
    CHK(lise_step(c, dt, 0));   // start-up if needed
    const long long per_bytes = c->per * (long long)c->esz;
    const long long gib = std::max<long long>(1, (1LL << 30) / std::max<long long>(per_bytes, 1));
    std::vector<long long> chunks = {std::min<long long>(c->M, gib), std::min<long long>(c->M, 2 * gib),
                                     std::min<long long>(c->M, 4 * gib),
                                     std::min<long long>(c->M, std::max<long long>(16, gib / 4))};
    std::sort(chunks.begin(), chunks.end());
    chunks.erase(std::unique(chunks.begin(), chunks.end()), chunks.end());
    const int jgs[] = {8, 16, 32, 64};
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    // time nsteps of the candidate t (after one untimed step in its shape)
    auto trial = [&](const lise_tuning& t, int nsteps, float* ms) {
        int r = lise_set_tuning(c, &t);
        if (r == LISE_OK) r = lise_step(c, dt, 1);
        if (r != LISE_OK) return r;
        (void)hipEventRecord(e0, c->stream);
        r = lise_step(c, dt, nsteps);
        (void)hipEventRecord(e1, c->stream);
        (void)hipEventSynchronize(e1);
        *ms = 0.0f;
        (void)hipEventElapsedTime(ms, e0, e1);
        return r;
    };
    // first pass: every candidate; second pass: the three fastest again over twice the
    // steps, so that timing noise between close candidates does not decide
    std::vector<std::pair<float, lise_tuning>> timed;
    int rc = LISE_OK;
    // the single-pass kernel where it applies (its chunk only splits launches;
    // no z kernel to overlap), then the two-kernel path
    const bool cube_ok = c->single_pass >= 0 && cube_eligible(c);   // both paths are candidates
    if (cube_ok) {
        const int cjgs[] = {2, 4, 8, 16};
        for (int jg : cjgs) {
            if (rc != LISE_OK) break;
            lise_tuning t{};
            t.chunk_qpwf = (int32_t)std::min<long long>(c->M, gib);
            t.jgroup = jg;
            t.fused = c->fused_mode;
            t.generic = c->generic;
            t.no_overlap = 1;
            t.graph = c->use_graph;
            t.single_pass = 1;
            t.z_dense = c->z_dense_user;
            float ms = 0.0f;
            rc = trial(t, trial_steps, &ms);
            if (rc == LISE_OK) timed.push_back({ms, t});
        }
    }
    // the plane kernel with the z-term inside (one launch per phase: no
    // chunk or overlap to choose)
    const bool zd_ok = c->z_dense_user >= 0 && zdense_eligible(c);
    if (zd_ok) {
        const int zjgs[] = {32, 64, 128, 256};
        for (int jg : zjgs) {
            if (rc != LISE_OK) break;
            lise_tuning t{};
            t.chunk_qpwf = (int32_t)std::min<long long>(c->M, gib);
            t.jgroup = jg;
            t.fused = c->fused_mode;
            t.generic = c->generic;
            t.no_overlap = 1;
            t.graph = c->use_graph;
            t.single_pass = -1;
            t.z_dense = 1;
            float ms = 0.0f;
            rc = trial(t, trial_steps, &ms);
            if (rc == LISE_OK) timed.push_back({ms, t});
        }
    }
    for (long long ch : chunks)
        for (int jg : jgs)
            for (int nov = 0; nov < 2 && rc == LISE_OK; ++nov) {
                if (c->fused && nov) continue;
                lise_tuning t{};
                t.chunk_qpwf = (int32_t)ch;
                t.jgroup = jg;
                t.fused = c->fused_mode;
                t.generic = c->generic;
                t.no_overlap = nov;
                t.graph = c->use_graph;
                t.single_pass = cube_ok ? -1 : c->single_pass;
                t.z_dense = zd_ok ? -1 : c->z_dense_user;
                float ms = 0.0f;
                rc = trial(t, trial_steps, &ms);
                if (rc == LISE_OK) timed.push_back({ms, t});
            }
    lise_tuning best{};
    if (rc == LISE_OK && !timed.empty()) {
        std::sort(timed.begin(), timed.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
        best = timed[0].second;
        float best_ms = 1e30f;
        // second round: the three fastest, each also with 2 and 4 lanes per
        // z-column where the z kernel runs (two-kernel path, lanes valid)
        std::vector<lise_tuning> second;
        for (size_t i = 0; i < std::min<size_t>(3, timed.size()); ++i) {
            lise_tuning t = timed[i].second;
            second.push_back(t);
            if (t.single_pass > 0 || t.z_dense > 0 || !c->fast_z) continue;
            for (int zl : {2, 4})
                if (kz_lanes_valid(c->lat.nz, zl)) {
                    t.z_lanes = zl;
                    second.push_back(t);
                }
        }
        for (size_t i = 0; i < second.size() && rc == LISE_OK; ++i) {
            float ms = 0.0f;
            rc = trial(second[i], 2 * trial_steps, &ms);
            if (rc == LISE_OK && ms < best_ms) {
                best_ms = ms;
                best = second[i];
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != LISE_OK) return rc;
    CHK(lise_set_tuning(c, &best));
    if (chosen) *chosen = best;
    return LISE_OK;
}

const char* lise_last_error(const lise_ctx* c) { return c ? c->err : "null context"; }

const char* lise_version(void) { return kVersion; }

int lise_kick(lise_ctx* c, const double* chi, int32_t chi_is_device) {
    if (!c || !chi) return LISE_E_ARG;
    if (c->n_set < c->M) return fail(c, LISE_E_STATE, "qpwfs not fully set");
    const double* cd = chi;
    if (!chi_is_device) {
        HIPCHK(c, hipMemcpyAsync(c->V_tmp, chi, (size_t)c->N * sizeof(double), hipMemcpyHostToDevice, c->stream));
        cd = c->V_tmp;
    }
    int rc = c->prec == LISE_FP64 ? kick_t<double>(c, cd) : kick_t<float>(c, cd);
    if (rc != LISE_OK) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // the state jumped: new densities, and the ABM history restarts
    c->hist = false;
    c->dens_valid = false;
    return LISE_OK;
}

int lise_current(lise_ctx* c, double* j_out, int32_t out_is_device) {
    if (!c || !j_out) return LISE_E_ARG;
    if (c->n_set < c->M) return fail(c, LISE_E_STATE, "qpwfs not fully set");
    double* dst = out_is_device ? j_out : c->dens_tmp;
    int rc = c->prec == LISE_FP64 ? current_t<double>(c, dst) : current_t<float>(c, dst);
    if (rc != LISE_OK) return rc;
    if (!out_is_device)
        HIPCHK(c, hipMemcpyAsync(j_out, dst, 3 * (size_t)c->N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LISE_OK;
}

int lise_coupling(const lise_lattice* lat, const lise_functional* fn, double* g_out) {
    if (!lat || !fn || !g_out) return LISE_E_ARG;
    if (fn->regularize != 0 && fn->regularize != 1) return LISE_E_ARG;
    return lise::plan::effective_coupling(fn->g, lat->a, fn->regularize, g_out) ? LISE_OK : LISE_E_ARG;
}

void lise_free(lise_ctx* c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    if (c->s2) (void)hipStreamSynchronize(c->s2);
    for (auto& p : c->buf) dfree(&p);
    dfree(&c->Gbuf[0]);
    dfree(&c->Gbuf[1]);
    c->G = nullptr;
    if (c->s2) (void)hipStreamDestroy(c->s2);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    if (c->ev_cap) (void)hipEventDestroy(c->ev_cap);
    if (c->ev_start) (void)hipEventDestroy(c->ev_start);
    for (int i = 0; i < 2; ++i) {
        if (c->ev_kz[i]) (void)hipEventDestroy(c->ev_kz[i]);
        if (c->ev_kp[i]) (void)hipEventDestroy(c->ev_kp[i]);
    }
    dfree(reinterpret_cast<void**>(&c->dpart));
    dfree(reinterpret_cast<void**>(&c->dens_cur));
    dfree(reinterpret_cast<void**>(&c->dens_tmp));
    dfree(reinterpret_cast<void**>(&c->V_cur));
    dfree(reinterpret_cast<void**>(&c->V_tmp));
    dfree(reinterpret_cast<void**>(&c->D_cur));
    dfree(reinterpret_cast<void**>(&c->D_tmp));
    dfree(&c->tw);
    dfree(reinterpret_cast<void**>(&c->red));
    dfree(&c->ah_buf);
    dfree(&c->cube_desc);
    dfree(&c->tzm);
    dfree(reinterpret_cast<void**>(&c->norms));
    dfree(reinterpret_cast<void**>(&c->norms0));
    dfree(reinterpret_cast<void**>(&c->eta));
    dfree(reinterpret_cast<void**>(&c->eta_part));
    dfree(reinterpret_cast<void**>(&c->pz_part));
    for (int b = 0; b < 2; ++b) dfree(reinterpret_cast<void**>(&c->ez_part[b]));
    dfree(reinterpret_cast<void**>(&c->bad));
    dfree(reinterpret_cast<void**>(&c->dtime));
    dfree(reinterpret_cast<void**>(&c->dkin));
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    for (auto& ev : c->prof.pool) (void)hipEventDestroy(ev);
    delete c;
}

}  // extern "C"

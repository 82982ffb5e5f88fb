// C ABI declared in include/sph.h.  The launch sequences live in
// sph_engine.hpp and are instantiated in sph_part.hip, one (dimension,
// kernel, pair precision) per translation unit.
#include "sph_engine.hpp"

using namespace sph_host;

#include <mutex>

// Static workspace of sph_step_noalloc: one copy per device.  Host code never
// passes this name to a kernel (in host code it is a stand-in, not a device
// address); it uses the address hipGetSymbolAddress returns for the current
// device, kept per device below.
static __device__ __align__(256) unsigned char scratch[SPH_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once).
int scratch_address(void** out) {
    int dev = 0;
    SPH_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SPH_EDEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        SPH_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(SPH_EDEVICE, "no device address for the static scratch");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SPH_OK;
}
}  // namespace

#define SPH_EXTERN_API(D, K, TT) extern template struct sph_host::Api<D, K, TT>;
SPH_FOR_EACH_COMBO(SPH_EXTERN_API)
#undef SPH_EXTERN_API

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

const char* sph_last_error(void) { return g_err.c_str(); }

int sph_grid(const sph_params* prm, int64_t nc[3], int64_t* ncells) {
    g_err.clear();
    SPH_TRY(check_params(prm, false));
    if (!nc || !ncells) return fail(SPH_EINVAL, "output pointer is NULL");
    sph::Grid G;
    SPH_TRY(make_grid(prm, &G, ncells));
    for (int k = 0; k < 3; ++k) nc[k] = G.nc[k];
    return SPH_OK;
}

size_t sph_workspace_bytes(const sph_params* prm, int64_t n, int64_t adjoint_k) {
    g_err.clear();
    if (check_params(prm, false) != SPH_OK) return 0;
    if (n < 1 || n >= ((int64_t)1 << 31) - sph::kScanChunk) {
        fail(SPH_EINVAL, "n out of range");
        return 0;
    }
    if (adjoint_k < 0) {
        fail(SPH_EINVAL, "adjoint_k must be >= 0");
        return 0;
    }
    sph::Grid G;
    int64_t ncells;
    if (make_grid(prm, &G, &ncells) != SPH_OK) return 0;
    return make_layout(prm, G, n, ncells, adjoint_k).bytes;
}

int sph_bin_sort(const sph_params* prm, sph_particles* pa, void* ws, size_t ws_bytes,
                 uint32_t* cell_start, uint32_t* cell_end, void* stream) {
    g_err.clear();
    SPH_TRY(check_params(prm, false));
    SPH_TRY(check_particles(prm, pa));
    if (!cell_start || !cell_end) return fail(SPH_EINVAL, "cell_start/cell_end is NULL");
    return dispatch(prm, [&](auto A) {
        return decltype(A)::bin_sort(prm, pa, ws, ws_bytes, cell_start, cell_end, stream);
    });
}

int sph_neighbors(const sph_params* prm, const sph_particles* pa, const uint32_t* cell_start,
                  const uint32_t* cell_end, int64_t capacity, int64_t* offsets, int32_t* nbr,
                  int64_t* total, void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    SPH_TRY(check_params(prm, false));
    SPH_TRY(check_particles(prm, pa));
    if (!cell_start || !cell_end || !offsets || !total)
        return fail(SPH_EINVAL, "cell ranges, offsets or total is NULL");
    if (capacity < 0) return fail(SPH_EINVAL, "capacity must be >= 0");
    return dispatch(prm, [&](auto A) {
        return decltype(A)::neighbors(prm, pa, cell_start, cell_end, capacity, offsets, nbr, total, ws,
                                  ws_bytes, stream);
    });
}

int sph_density(const sph_params* prm, sph_particles* pa, const uint32_t* cell_start,
                const uint32_t* cell_end, void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    SPH_TRY(check_params(prm, false));
    SPH_TRY(check_particles(prm, pa));
    if (!cell_start || !cell_end) return fail(SPH_EINVAL, "cell_start/cell_end is NULL");
    return dispatch(prm, [&](auto A) {
        return decltype(A)::density(prm, pa, cell_start, cell_end, ws, ws_bytes, stream);
    });
}

int sph_eos(const sph_params* prm, sph_particles* pa, void* stream) {
    g_err.clear();
    SPH_TRY(check_params(prm, false));
    if (!pa || pa->n < 1 || pa->n >= ((int64_t)1 << 31) || !pa->rho || !pa->p)
        return fail(SPH_EINVAL, "need n >= 1 and rho, p");
    return dispatch(prm, [&](auto A) {
        return decltype(A)::eos(prm, pa, stream);
    });
}

int sph_momentum(const sph_params* prm, sph_particles* pa, const uint32_t* cell_start,
                 const uint32_t* cell_end, void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    SPH_TRY(check_params(prm, false));
    SPH_TRY(check_particles(prm, pa));
    if (!cell_start || !cell_end) return fail(SPH_EINVAL, "cell_start/cell_end is NULL");
    return dispatch(prm, [&](auto A) {
        return decltype(A)::momentum(prm, pa, cell_start, cell_end, ws, ws_bytes, stream);
    });
}

int sph_step(const sph_params* prm, sph_particles* pa, int64_t nsteps, int prime_accel, void* ws,
             size_t ws_bytes, double* diag, void* stream) {
    g_err.clear();
    SPH_TRY(check_params(prm, true));
    SPH_TRY(check_particles(prm, pa));
    if (nsteps < 0) return fail(SPH_EINVAL, "nsteps must be >= 0");
    if (prime_accel != 0 && prime_accel != 1) return fail(SPH_EINVAL, "prime_accel must be 0 or 1");
    return dispatch(prm, [&](auto A) {
        return decltype(A)::step(prm, pa, nsteps, prime_accel, ws, ws_bytes, diag, stream);
    });
}

int sph_step_noalloc(const sph_params* prm, sph_particles* pa, int64_t nsteps, int prime_accel,
                     double* diag, void* stream) {
    g_err.clear();
    SPH_TRY(check_params(prm, true));
    SPH_TRY(check_particles(prm, pa));
    if (nsteps < 0) return fail(SPH_EINVAL, "nsteps must be >= 0");
    if (prime_accel != 0 && prime_accel != 1) return fail(SPH_EINVAL, "prime_accel must be 0 or 1");
    sph::Grid G;
    int64_t ncells;
    SPH_TRY(make_grid(prm, &G, &ncells));
    const Layout L = make_layout(prm, G, pa->n, ncells, 0);
    if (L.bytes > SPH_NOALLOC_SCRATCH_BYTES)
        return fail(SPH_EWORKSPACE, "the step needs %zu bytes of workspace, the static scratch holds %zu",
                    L.bytes, (size_t)SPH_NOALLOC_SCRATCH_BYTES);
    void* ws = nullptr;
    SPH_TRY(scratch_address(&ws));
    // the flag words and interaction counters start at zero (a fill kernel,
    // so that the call can be captured into a graph)
    hipStream_t st = (hipStream_t)stream;
    const int64_t words = (int64_t)(L.counts / 4);
    launch(K_FILL, sph::k_fill_u32, blocks_for(words), st, words, 0u, (uint32_t*)ws);
    SPH_TRY(launch_check("k_fill_u32"));
    return dispatch(prm, [&](auto A) {
        return decltype(A)::step(prm, pa, nsteps, prime_accel, ws, (size_t)SPH_NOALLOC_SCRATCH_BYTES,
                                 diag, stream);
    });
}

int sph_step_backward(const sph_params* prm, const sph_particles* ckpt, int64_t k,
                      const double* lam_in, double* lam_out, double* dJ_dnu, void* ws,
                      size_t ws_bytes, void* stream) {
    g_err.clear();
    SPH_TRY(check_params(prm, true));
    SPH_TRY(check_particles(prm, ckpt));
    if (k < 1) return fail(SPH_EINVAL, "k must be >= 1");
    if (!lam_in || !lam_out || !dJ_dnu) return fail(SPH_EINVAL, "lam_in, lam_out or dJ_dnu is NULL");
    if (lam_in == lam_out) return fail(SPH_EINVAL, "lam_in and lam_out may not alias");
    if (prm->scheme != SPH_SCHEME_SUMMATION)
        return fail(SPH_EINVAL, "the adjoint covers the summation scheme only");
    return dispatch(prm, [&](auto A) {
        return decltype(A)::step_backward(prm, ckpt, k, lam_in, lam_out, dJ_dnu, ws, ws_bytes, stream);
    });
}

int sph_ke_seed(const sph_params* prm, const sph_particles* pa, double scale, double* lam,
                void* stream) {
    g_err.clear();
    SPH_TRY(check_params(prm, false));
    SPH_TRY(check_particles(prm, pa));
    if (!lam) return fail(SPH_EINVAL, "lam is NULL");
    if (!std::isfinite(scale)) return fail(SPH_EINVAL, "scale must be finite");
    hipStream_t st = (hipStream_t)stream;
    const int n = (int)pa->n;
    if (prm->dim == 2)
        launch(K_ADJ_SEED, sph::k_ke_seed<2>, blocks_for(n), st, n, (const double*)pa->u[0],
               (const double*)pa->u[1], (const double*)nullptr, (const double*)pa->m, scale, lam);
    else
        launch(K_ADJ_SEED, sph::k_ke_seed<3>, blocks_for(n), st, n, (const double*)pa->u[0],
               (const double*)pa->u[1], (const double*)pa->u[2], (const double*)pa->m, scale, lam);
    return launch_check("k_ke_seed");
}

int sph_accel_backward(const sph_params* prm, const sph_particles* st, const double* lam_a,
                       double* lam_x, double* lam_u, double* dJ_dnu, void* ws, size_t ws_bytes,
                       void* stream) {
    g_err.clear();
    SPH_TRY(check_params(prm, false));
    SPH_TRY(check_particles(prm, st));
    if (!lam_a || !lam_x || !lam_u || !dJ_dnu)
        return fail(SPH_EINVAL, "lam_a, lam_x, lam_u or dJ_dnu is NULL");
    if (prm->scheme != SPH_SCHEME_SUMMATION)
        return fail(SPH_EINVAL, "the adjoint covers the summation scheme only");
    return dispatch(prm, [&](auto A) {
        return decltype(A)::accel_backward(prm, st, lam_a, lam_x, lam_u, dJ_dnu, ws, ws_bytes, stream);
    });
}

int sph_read_interactions(void* ws, size_t ws_bytes, int64_t* total, int reset, void* stream) {
    g_err.clear();
    if (!ws || ws_bytes < 256 || !total) return fail(SPH_EINVAL, "workspace or total is NULL");
    hipStream_t st = (hipStream_t)stream;
    unsigned long long nb = 0;
    SPH_HIP(hipMemcpyAsync(&nb, (char*)ws + 8, sizeof nb, hipMemcpyDeviceToHost, st));
    SPH_HIP(hipStreamSynchronize(st));
    *total = 0;
    if (nb == 0) return SPH_OK;  // no density evaluation yet
    if (16 + 8 * nb > ws_bytes) return fail(SPH_EINVAL, "corrupt interaction counter header");
    std::vector<unsigned long long> v(nb);
    SPH_HIP(hipMemcpyAsync(v.data(), (char*)ws + 16, 8 * nb, hipMemcpyDeviceToHost, st));
    SPH_HIP(hipStreamSynchronize(st));
    unsigned long long t = 0;
    for (unsigned long long x : v) t += x;
    *total = (int64_t)t;
    if (reset) {
        SPH_HIP(hipMemsetAsync((char*)ws + 16, 0, 8 * nb, st));
        SPH_HIP(hipStreamSynchronize(st));
    }
    return SPH_OK;
}

int sph_timer_enable(int on) {
    g_err.clear();
    if (on != 0 && on != 1) return fail(SPH_EINVAL, "on must be 0 or 1");
    g_timer.on = on != 0;
    return SPH_OK;
}

int sph_timer_read(int nslots, const char** names, double* ms, int64_t* launches, int reset) {
    g_err.clear();
    g_timer.fold();
    for (int k = 0; k < nslots && k < K_COUNT; ++k) {
        if (names) names[k] = kKernelNames[k];
        if (ms) ms[k] = g_timer.ms[k];
        if (launches) launches[k] = g_timer.launches[k];
    }
    if (reset) {
        for (int k = 0; k < K_COUNT; ++k) {
            g_timer.ms[k] = 0.0;
            g_timer.launches[k] = 0;
        }
    }
    return K_COUNT;
}

int sph_check(void* ws, size_t ws_bytes, void* stream) {
    g_err.clear();
    if (!ws || ws_bytes < 256) return fail(SPH_EINVAL, "workspace is NULL or too small");
    hipStream_t st = (hipStream_t)stream;
    uint32_t flags = 0;
    SPH_HIP(hipMemcpyAsync(&flags, ws, sizeof flags, hipMemcpyDeviceToHost, st));
    SPH_HIP(hipStreamSynchronize(st));
    if (flags) {
        SPH_HIP(hipMemsetAsync(ws, 0, sizeof flags, st));
        SPH_HIP(hipStreamSynchronize(st));
    }
    if (flags & sph::kFlagNonFinite) return fail(SPH_ENONFINITE, "non-finite position or velocity");
    if (flags & sph::kFlagOutside)
        return fail(SPH_EDOMAIN, "particle outside a non-periodic domain (clamped to edge cells)");
    return SPH_OK;
}

}  // extern "C"

// dry.hip -- optional dry attributes of the super-droplets (Sect. 5.1.4: on
// coalescence, extensive particle parameters such as the dry radius cubed are
// summed and intensive ones such as the hygroscopicity kappa averaged).
//
// Attached to a context, they live in storage order in a caller-owned
// workspace; the coalescence step (merge_dry), recycling and the transport
// re-sort keep them with their particles.  Dry-radius moments use the
// correctly rounded cube root of r_d^3.
#include "context.hpp"
#include "diag_kernels.hpp"

#include <cmath>

using namespace sdm;

namespace {

constexpr unsigned int kErrDry = 8u;

// storage slot s <- input index id[s]; r_d^3 must be finite and > 0, kappa finite and >= 0
__global__ void k_dry_in(uint64_t n, const uint32_t* __restrict__ id,
                         const double* __restrict__ rd3_in, const double* __restrict__ kappa_in,
                         double* __restrict__ rd3, double* __restrict__ kappa,
                         unsigned int* __restrict__ err)
{
    for (uint64_t s = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; s < n;
         s += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const double v = rd3_in[id[s]], k = kappa_in[id[s]];
        if (!(v > 0.0 && v < __builtin_inf()) || !(k >= 0.0 && k < __builtin_inf()))
            atomicOr(err, kErrDry);
        rd3[s] = v;
        kappa[s] = k;
    }
}

__global__ void k_dry_out(uint64_t n, const uint32_t* __restrict__ id,
                          const double* __restrict__ rd3, const double* __restrict__ kappa,
                          double* __restrict__ rd3_out, double* __restrict__ kappa_out)
{
    for (uint64_t s = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; s < n;
         s += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        if (rd3_out) rd3_out[id[s]] = rd3[s];
        if (kappa_out) kappa_out[id[s]] = kappa[s];
    }
}

struct DryLayout {
    double *rd3, *kappa, *rd3_alt, *kappa_alt;
    size_t bytes;
};

DryLayout dry_layout(void* ws, size_t ws_bytes, uint64_t n)
{
    Carver cv(ws, ws_bytes);
    DryLayout L{};
    L.rd3 = cv.take<double>(n);
    L.kappa = cv.take<double>(n);
    L.rd3_alt = cv.take<double>(n);
    L.kappa_alt = cv.take<double>(n);
    L.bytes = cv.used();
    return L;
}

sdm_status check_dry(const sdm_ctx* x)
{
    if (!x) {
        set_error("context is NULL");
        return SDM_EINVAL;
    }
    if (!x->rd3) {
        set_error("no dry attributes attached (sdm_dry_attach)");
        return SDM_ESTATE;
    }
    return SDM_OK;
}

}  // namespace

extern "C" size_t sdm_dry_workspace_bytes(uint64_t n_sd)
{
    return dry_layout(nullptr, 0, n_sd).bytes;
}

extern "C" sdm_status sdm_dry_attach(sdm_ctx* x, void* workspace, size_t ws_bytes,
                                     const double* rd3_in, const double* kappa_in)
{
    if (!x) {
        set_error("context is NULL");
        return SDM_EINVAL;
    }
    if (x->rd3) {
        set_error("dry attributes are already attached");
        return SDM_ESTATE;
    }
    if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255u)) {
        set_error("workspace must be non-NULL and 256-byte aligned");
        return SDM_EINVAL;
    }
    const uint64_t n = x->n_sd;
    if (n > 0 && (!rd3_in || !kappa_in)) {
        set_error("rd3 and kappa must be non-NULL");
        return SDM_EINVAL;
    }
    const DryLayout L = dry_layout(workspace, ws_bytes, n);
    if (L.bytes > ws_bytes) {
        set_error("dry workspace has %zu bytes, %zu needed", ws_bytes, L.bytes);
        return SDM_ENOMEM;
    }
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, x->stream,
                       reinterpret_cast<uint32_t*>(x->err), uint64_t(1), 0u);
    SDM_LAUNCHED();
    if (n > 0) {
        hipLaunchKernelGGL(k_dry_in, dim3(grid_for(n, 256, 8192)), dim3(256), 0, x->stream, n,
                           x->id, rd3_in, kappa_in, L.rd3, L.kappa, x->err);
        SDM_LAUNCHED();
    }
    unsigned int err = 0;
    SDM_HIP(hipMemcpyAsync(&err, x->err, sizeof(err), hipMemcpyDeviceToHost, x->stream));
    SDM_HIP(hipStreamSynchronize(x->stream));
    if (err & kErrDry) {
        set_error("rd3 must be finite and > 0, kappa finite and >= 0");
        return SDM_EINVAL;
    }
    x->rd3 = L.rd3;
    x->kappa = L.kappa;
    x->rd3_alt = L.rd3_alt;
    x->kappa_alt = L.kappa_alt;
    return SDM_OK;
}

extern "C" sdm_status sdm_dry_get(sdm_ctx* x, double* rd3_out, double* kappa_out)
{
    SDM_TRY(check_dry(x));
    const uint64_t n = x->n_sd;
    if (n > 0 && (rd3_out || kappa_out)) {
        hipLaunchKernelGGL(k_dry_out, dim3(grid_for(n, 256, 8192)), dim3(256), 0, x->stream, n,
                           x->id, x->rd3, x->kappa, rd3_out, kappa_out);
        SDM_LAUNCHED();
    }
    SDM_HIP(hipStreamSynchronize(x->stream));
    return SDM_OK;
}

extern "C" sdm_status sdm_diag_dry_moments(sdm_ctx* x, uint32_t k, double rd_min, double rd_max,
                                           const double* rho_d, double* out)
{
    SDM_TRY(check_dry(x));
    if (k > kMaxMomentOrder) {
        set_error("moment order %u above %u", k, kMaxMomentOrder);
        return SDM_EINVAL;
    }
    if (std::isnan(rd_min) || std::isnan(rd_max)) {
        set_error("radius range bounds must not be NaN");
        return SDM_EINVAL;
    }
    if (x->n_cells == 0) return SDM_OK;
    if (!out) {
        set_error("out must be non-NULL");
        return SDM_EINVAL;
    }
    hipLaunchKernelGGL(k_moments<true>, dim3(grid_for(x->n_cells, kDiagCellsPerBlock, kDiagMaxBlocks)),
                       dim3(kDiagBlock), 0, x->stream, x->offsets, x->dV, x->xi, x->rd3,
                       x->n_cells, k, rd_min, rd_max, rho_d, out);
    SDM_LAUNCHED();
    return SDM_OK;
}

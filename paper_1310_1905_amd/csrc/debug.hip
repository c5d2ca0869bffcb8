// debug.hip -- element-wise entry points that run the step's device
// arithmetic (Philox, cube root, one collision test) on arrays, so that the
// parity tests can compare each piece with the CPU oracle bit for bit.
#include "runtime.hpp"

#include <cmath>

using namespace sdm;

namespace {

__global__ void k_debug_philox(uint64_t n, const uint32_t* ctr, const uint32_t* key, uint32_t* out)
{
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const Words4 w = philox4x32_10(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3],
                                       key[2 * i], key[2 * i + 1]);
        for (int t = 0; t < 4; ++t) out[4 * i + t] = w.w[t];
    }
}

__global__ void k_debug_cbrt(uint64_t n, const double* x, double* y)
{
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        y[i] = cbrt_rn(x[i]);
}

__global__ void k_debug_collide(uint64_t n, uint32_t kind, KernelParams kp, double dt,
                                const uint32_t* n_live, const double* dV, const double* u,
                                uint64_t* xi_a, double* r_a, uint64_t* xi_b, double* r_b,
                                double* K_out, double* p_out, uint64_t* gamma_out)
{
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint64_t xa = xi_a[i], xb = xi_b[i];
        const double ra = r_a[i], rb = r_b[i];
        const double K = collection_kernel(kind, kp, ra, rb);
        const bool a_is_j = xa >= xb;
        PairState s;
        s.xj = a_is_j ? xa : xb;
        s.xk = a_is_j ? xb : xa;
        s.rj = a_is_j ? ra : rb;
        s.rk = a_is_j ? rb : ra;
        const double p = collision_probability(s.xj, K, dt, dV[i], upscale_factor(n_live[i]));
        const uint64_t g = collision_count(p, u[i], s.xj, s.xk);
        if (g > 0) apply_collisions(g, s);
        K_out[i] = K;
        p_out[i] = p;
        gamma_out[i] = g;
        xi_a[i] = a_is_j ? s.xj : s.xk;
        xi_b[i] = a_is_j ? s.xk : s.xj;
        r_a[i] = a_is_j ? s.rj : s.rk;
        r_b[i] = a_is_j ? s.rk : s.rj;
    }
}

// Philox over a counter range: element i takes counter (c0 + lo32(i),
// c1 + hi32(i), c2, c3) (each word modulo 2^32) and key (k0, k1).
__global__ void k_debug_philox_range(uint64_t n, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1, uint32_t* out)
{
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const Words4 w = philox4x32_10(c0 + static_cast<uint32_t>(i),
                                       c1 + static_cast<uint32_t>(i >> 32), c2, c3, k0, k1);
        uint4 v;
        v.x = w.w[0];
        v.y = w.w[1];
        v.z = w.w[2];
        v.w = w.w[3];
        reinterpret_cast<uint4*>(out)[i] = v;
    }
}

// The square root of the terminal velocity's top branch (v_t = k3 sqrt(r) with
// k3 = 1) and the division of eq. (P_ij) (p = ((xi K) dt / dV) scale with
// xi = dt = scale = 1, K = a, dV = b): both through the step's own functions.
__global__ void k_debug_sqrt_div(uint64_t n, const double* a, const double* b, double* sq,
                                 double* q)
{
    KernelParams kp{};
    kp.k3 = 1.0;
    kp.r1 = 0.0;
    kp.r2 = 0.0;
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const double x = a[i];
        if (sq) sq[i] = terminal_velocity(kp, x);
        if (q) q[i] = collision_probability(1u, x, 1.0, b[i], 1.0);
    }
}

}  // namespace

extern "C" sdm_status sdm_debug_philox_range(void* stream, uint64_t n, const uint32_t* counter,
                                             const uint32_t* key, uint32_t* out)
{
    if (n == 0) return SDM_OK;
    if (!counter || !key || !out) {
        set_error("NULL array");
        return SDM_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_debug_philox_range, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, n,
                       counter[0], counter[1], counter[2], counter[3], key[0], key[1], out);
    SDM_LAUNCHED();
    SDM_HIP(hipStreamSynchronize(s));
    return SDM_OK;
}

extern "C" sdm_status sdm_debug_sqrt_div(void* stream, uint64_t n, const double* a,
                                         const double* b, double* sqrt_out, double* div_out)
{
    if (n == 0) return SDM_OK;
    if (!a || (div_out && !b) || (!sqrt_out && !div_out)) {
        set_error("NULL array");
        return SDM_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_debug_sqrt_div, dim3(grid_for(n, 256, 16384)), dim3(256), 0, s, n, a, b,
                       sqrt_out, div_out);
    SDM_LAUNCHED();
    SDM_HIP(hipStreamSynchronize(s));
    return SDM_OK;
}

extern "C" sdm_status sdm_debug_philox(void* stream, uint64_t n, const uint32_t* ctr,
                                       const uint32_t* key, uint32_t* out)
{
    if (n == 0) return SDM_OK;
    if (!ctr || !key || !out) {
        set_error("NULL array");
        return SDM_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_debug_philox, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, ctr, key,
                       out);
    SDM_LAUNCHED();
    SDM_HIP(hipStreamSynchronize(s));
    return SDM_OK;
}

extern "C" sdm_status sdm_debug_cbrt(void* stream, uint64_t n, const double* x, double* y)
{
    if (n == 0) return SDM_OK;
    if (!x || !y) {
        set_error("NULL array");
        return SDM_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_debug_cbrt, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n, x, y);
    SDM_LAUNCHED();
    SDM_HIP(hipStreamSynchronize(s));
    return SDM_OK;
}

extern "C" sdm_status sdm_debug_collide(void* stream, uint64_t n, sdm_kernel kernel,
                                        const sdm_kernel_params* params, double dt,
                                        const uint32_t* n_live, const double* dV, const double* u,
                                        uint64_t* xi_a, double* r_a, uint64_t* xi_b, double* r_b,
                                        double* K_out, double* p_out, uint64_t* gamma_out)
{
    if (n == 0) return SDM_OK;
    if (!n_live || !dV || !u || !xi_a || !r_a || !xi_b || !r_b || !K_out || !p_out || !gamma_out) {
        set_error("NULL array");
        return SDM_EINVAL;
    }
    if (kernel != SDM_KERNEL_GOLOVIN && kernel != SDM_KERNEL_GEOMETRIC) {
        set_error("unknown kernel");
        return SDM_EINVAL;
    }
    sdm_kernel_params kp;
    sdm_default_params(&kp);
    if (params) kp = *params;
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(k_debug_collide, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, n,
                       static_cast<uint32_t>(kernel), to_kp(kp), dt, n_live, dV, u, xi_a, r_a, xi_b,
                       r_b, K_out, p_out, gamma_out);
    SDM_LAUNCHED();
    SDM_HIP(hipStreamSynchronize(s));
    return SDM_OK;
}

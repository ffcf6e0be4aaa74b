// Velocity-Verlet NVE molecular dynamics driven by the D3 forces.  Each
// step: half kick and drift, forces at the new positions (neighbour lists
// rebuilt when an atom moved more than half the skin), second half kick.
// Units: Angstrom, fs, amu, eV.
#include <vector>

#include "d3_ctx.h"

namespace d3 {

// 1 eV / (Angstrom amu) in Angstrom / fs^2, and 1 amu Angstrom^2 / fs^2 in eV
constexpr double ACC_UNIT = 9.648533212331e-3;
constexpr double KE_UNIT = 103.642691;

__global__ void __launch_bounds__(BLOCK)
k_kick_drift(int n, double dt, double* __restrict__ pos, double* __restrict__ vel,
             const double* __restrict__ f, const double* __restrict__ mass, int drift)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = 0.5 * dt * ACC_UNIT / mass[i];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const double v = vel[3 * i + k] + a * f[3 * i + k];
        vel[3 * i + k] = v;
        if (drift) pos[3 * i + k] += dt * v;
    }
}

// kinetic energy: per-workgroup partial sums, then one workgroup sums them
// in a fixed order
__global__ void __launch_bounds__(BLOCK)
k_ke_part(int n, const double* __restrict__ vel, const double* __restrict__ mass,
          double* __restrict__ part)
{
    __shared__ double sh[BLOCK];
    double s = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const double vx = vel[3 * i], vy = vel[3 * i + 1], vz = vel[3 * i + 2];
        s += mass[i] * (vx * vx + vy * vy + vz * vz);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = BLOCK / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void __launch_bounds__(BLOCK)
k_ke_final(int nparts, const double* __restrict__ part, double* __restrict__ out)
{
    __shared__ double sh[BLOCK];
    double s = 0.0;
    for (int b = threadIdx.x; b < nparts; b += BLOCK) s += part[b];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = BLOCK / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = 0.5 * KE_UNIT * sh[0];
}

}  // namespace d3

using namespace d3;

extern "C" int d3_md_nve(d3_ctx* c, int64_t n_steps, double dt, double* pos, double* vel,
                         const double* mass, int32_t every, double* thermo, int64_t* rebuilds,
                         void* stream)
{
    if (!c) return fail(D3_ERR_INVALID_ARG, "ctx is NULL");
    if (!c->built) return fail(D3_ERR_STATE, "d3_md_nve before d3_build_neighbors");
    if (n_steps < 0 || !(dt > 0.0) || every < 0 || (every > 0 && !thermo))
        return fail(D3_ERR_INVALID_ARG, "bad MD arguments");
    const int n = (int)c->n;
    if (n > 0 && (!pos || !vel || !mass)) return fail(D3_ERR_INVALID_ARG, "NULL buffer");
    hipStream_t s = (hipStream_t)stream;
    c->last_stream = s;
    const int nb = (n + BLOCK - 1) / BLOCK;
    const int kparts = nb < 1024 ? (nb > 0 ? nb : 1) : 1024;
    // scratch: forces (3n), energy (1), kinetic energy (1), KE partials
    const size_t need = ((size_t)3 * (n > 0 ? n : 1) + 2 + kparts) * sizeof(double);
    int r = ensure(c->md_scratch, need);
    if (r) return r;
    double* F = c->md_scratch.as<double>();
    double* E = F + 3 * (size_t)(n > 0 ? n : 1);
    double* K = E + 1;
    double* part = K + 1;
    const int64_t reb0 = c->n_rebuilds;
    auto record = [&](int64_t slot) -> int {
        hipLaunchKernelGGL(k_ke_part, dim3(kparts), dim3(BLOCK), 0, s, n, vel, mass, part);
        hipLaunchKernelGGL(k_ke_final, dim3(1), dim3(BLOCK), 0, s, kparts, part, K);
        double ek[2];
        hipError_t e = hipMemcpyAsync(ek, E, 2 * sizeof(double), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "md thermo");
        thermo[3 * slot] = ek[0];
        thermo[3 * slot + 1] = ek[1];
        thermo[3 * slot + 2] = ek[0] + ek[1];
        return D3_OK;
    };
    r = d3_energy_forces_virial(c, pos, E, F, nullptr, nullptr, D3_AUTO_REBUILD, stream);
    if (r) return r;
    if (every > 0 && (r = record(0))) return r;
    for (int64_t st = 1; st <= n_steps; st++) {
        if (n > 0)
            hipLaunchKernelGGL(k_kick_drift, dim3(nb), dim3(BLOCK), 0, s, n, dt, pos, vel, F, mass, 1);
        r = d3_energy_forces_virial(c, pos, E, F, nullptr, nullptr, D3_AUTO_REBUILD, stream);
        if (r) return r;
        if (n > 0)
            hipLaunchKernelGGL(k_kick_drift, dim3(nb), dim3(BLOCK), 0, s, n, dt, pos, vel, F, mass, 0);
        if (every > 0 && st % every == 0 && (r = record(st / every))) return r;
    }
    if (rebuilds) *rebuilds = c->n_rebuilds - reb0;
    // conditions recorded on the device during the run (a species index or
    // a position that was not finite); stale lists and overflows were
    // handled by the rebuilds
    int st = 0;
    r = read_status(c, s, &st);
    if (r) return r;
    hipError_t e = hipMemsetAsync(c->status.p, 0, sizeof(int), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "d3_md_nve");
    return status_code(st);
}

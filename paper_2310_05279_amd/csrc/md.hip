// Velocity-Verlet NVE molecular dynamics driven by the D3 forces.  Each
// step: half kick and drift, forces at the new positions (neighbour lists
// rebuilt when an atom moved more than half the skin), second half kick.
// Units: Angstrom, fs, amu, eV.
#include <algorithm>
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

// a device-decided rebuild ran this step: count it and clear the flag
__global__ void k_rebuilt(int* __restrict__ need, unsigned long long* __restrict__ count)
{
    if (threadIdx.x == 0 && blockIdx.x == 0 && *need) {
        *count += 1;
        *need = 0;
    }
}

}  // namespace d3

using namespace d3;

// Steps between the synchronisations that check the device conditions
// (list overflow, bad species or positions) and save a restart point.
constexpr int64_t MD_CHECK = 16;

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
    const size_t N = (size_t)(n > 0 ? n : 1);
    // scratch: forces (3n), energy, kinetic energy, KE partials, the restart
    // point (positions, velocities, forces: 9n), then the rebuild flag and count
    const size_t nd = 3 * N + 2 + (size_t)kparts + 9 * N;
    const size_t need_bytes = nd * sizeof(double) + 2 * sizeof(unsigned long long);
    int r = ensure(c->md_scratch, need_bytes);
    if (r) return r;
    double* F = c->md_scratch.as<double>();
    double* E = F + 3 * N;
    double* K = E + 1;
    double* part = K + 1;
    double* snap = part + kparts;
    int* flag = (int*)(snap + 9 * N);
    unsigned long long* count = (unsigned long long*)(flag + 2);
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
    // copy between the state (positions, velocities, forces) and the restart point
    auto save = [&](bool restore) -> int {
        const size_t b = 3 * N * sizeof(double);
        const hipMemcpyKind k = hipMemcpyDeviceToDevice;
        hipError_t e = restore ? hipMemcpyAsync(pos, snap, b, k, s) : hipMemcpyAsync(snap, pos, b, k, s);
        if (e == hipSuccess)
            e = restore ? hipMemcpyAsync(vel, snap + 3 * N, b, k, s)
                        : hipMemcpyAsync(snap + 3 * N, vel, b, k, s);
        if (e == hipSuccess)
            e = restore ? hipMemcpyAsync(F, snap + 6 * N, b, k, s)
                        : hipMemcpyAsync(snap + 6 * N, F, b, k, s);
        return e == hipSuccess ? D3_OK : hip_fail(e, "md restart point");
    };
    // step 0: forces at the starting positions (rebuilding the lists if
    // they are stale): the one synchronising evaluation
    r = d3_energy_forces_virial(c, pos, E, F, nullptr, nullptr, D3_AUTO_REBUILD, stream);
    if (r) return r;
    if (every > 0 && (r = record(0))) return r;
    if (n_steps == 0) {
        if (rebuilds) *rebuilds = c->n_rebuilds - reb0;
        return D3_OK;
    }
    HIPCHK(hipMemsetAsync(flag, 0, 2 * sizeof(unsigned long long), s));
    if ((r = save(false))) return r;
    const double hs = 0.5 * c->prm.skin;
    int64_t snap_step = 0;
    int rollbacks = 0, sticky = 0;
    // Each step: half kick and drift; the positions into the sorted layout,
    // an atom beyond half the skin raising the device flag; a rebuild that
    // runs only if the flag is raised (decided on the device: no host
    // synchronisation); forces; second half kick.  Every MD_CHECK steps (and
    // at thermo records and the end) the stream is synchronised: a list
    // overflow restarts from the last restart point with grown lists.
    for (int64_t st = 1; st <= n_steps; st++) {
        if (n > 0) {
            hipLaunchKernelGGL(k_kick_drift, dim3(nb), dim3(BLOCK), 0, s, n, dt, pos, vel, F, mass, 1);
            launch_update(n, pos, c->perm.as<int>(), c->shift_s.as<double4>(),
                          c->ref_s.as<double4>(), c->pos_s.as<double4>(), hs * hs,
                          c->status.as<int>(), flag, 1, s);
            if ((r = run_build(c, pos, c->type_copy.as<int32_t>(), false, s, flag))) return r;
            hipLaunchKernelGGL(k_rebuilt, dim3(1), dim3(WAVE), 0, s, flag, count);
            if ((r = evaluate(c, c->prm.mode, E, F, nullptr, nullptr, nullptr, nullptr, nullptr,
                              0, s)))
                return r;
            hipLaunchKernelGGL(k_kick_drift, dim3(nb), dim3(BLOCK), 0, s, n, dt, pos, vel, F, mass, 0);
            HIPCHK(hipGetLastError());
        }
        const bool rec = every > 0 && st % every == 0;
        if (!(rec || st % MD_CHECK == 0 || st == n_steps)) continue;
        int bits = 0;
        if ((r = read_status(c, s, &bits))) return r;
        HIPCHK(hipMemsetAsync(c->status.p, 0, sizeof(int), s));
        if (bits & ST_CAPACITY) {
            // lists overflowed since the restart point: redo those steps
            if (++rollbacks > 8)
                return fail(D3_ERR_CAPACITY, "neighbour lists overflowed repeatedly during MD");
            // the lists of the replay hold at least the counts that overflowed
            int mc[8];
            if ((r = list_stats(c, s, mc))) return r;
            c->min_cap_p = std::max(c->min_cap_p, mc[0] + std::max(16, mc[0] / 4));
            c->min_cap_c = std::max(c->min_cap_c, mc[1] + std::max(16, mc[1] / 4));
            if ((r = save(true))) return r;
            HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), s));
            c->lists_bad = true;  // the next build sizes the lists again
            if ((r = rebuild_grow(c, pos, s))) return r;
            st = snap_step;
            continue;
        }
        sticky |= bits & (ST_SPECIES | ST_NONFINITE);
        if (rec && (r = record(st / every))) return r;
        if ((r = save(false))) return r;
        snap_step = st;
    }
    unsigned long long dev_rebuilds = 0;
    HIPCHK(hipMemcpyAsync(&dev_rebuilds, count, sizeof(dev_rebuilds), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (rebuilds) *rebuilds = c->n_rebuilds - reb0 + (int64_t)dev_rebuilds;
    return status_code(sticky);
}

// Modified Gram-Schmidt for one Arnoldi column with the work vector resident
// in registers (Sec. 2.2.2, modified Arnoldi).
//
// The column's passes h_ij = <v_i, w>, w <- w - h_ij v_i (i = 0..j) and the
// norm h_{j+1,j} = ||w|| are dependent global reductions.  Launched as one
// kernel per pass, each pass streams w in and out (4 vectors of traffic);
// here one cooperative kernel keeps w in registers for the whole column, so a
// pass reads only v_i, and the blocks meet at an in-kernel barrier after each
// partial sum.
//
// Summation order is the canonical one of the per-pass kernels: thread t of
// the grid (256 blocks x 1024 threads = 262144 lanes) is lane t, it adds the
// elements t, t + T, t + 2T, ... in index order, each group of 256
// consecutive lanes is combined by the halving tree into one of 1024
// partials, and every block finishes the sum from all 1024 partials in the
// same order, so all blocks hold bit-identical h_ij.
//
// Cross-block traffic inside the kernel is limited to the 1024 partials and
// the barrier counters, all accessed with agent-scope atomics (coherent
// across XCDs without an L2 write-back); every spin is bounded and reports a
// status flag instead of hanging.
#include "rok.h"
#include "rok_device.hpp"
#include "rok_kernels.hpp"

namespace rok {

constexpr int kPT = 1024;                       // threads per block
constexpr int kPB = kRedBlocks * kRedThreads / kPT;  // 256 blocks
constexpr double kBreakdownTolR = 1e-13;
constexpr long kSpinLimit = 1L << 22;

#define AGENT __HIP_MEMORY_SCOPE_AGENT

// Grid barrier, two levels: the blocks are split into kBarGroups groups;
// the last arrival of a group bumps the top counter, the last arrival at the
// top bumps the generation everyone waits on.  Counters sit on separate
// 128-byte lines.  bar (unsigned): [g * 32] group g arrivals, [kBarTop] top
// arrivals, [kBarGen] generation, [kBarErr] error.  Returns true (in every
// thread of the block) if the barrier failed.
constexpr int kBarGroups = 16;
constexpr int kBarTop = kBarGroups * 32;
constexpr int kBarGen = kBarTop + 32;
constexpr int kBarErr = kBarGen + 32;

__device__ __forceinline__ bool grid_sync(unsigned* bar) {
    __shared__ unsigned s_err;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned per_group = gridDim.x / kBarGroups;
        const unsigned grp = blockIdx.x / per_group;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        unsigned g = __hip_atomic_load(bar + kBarGen, __ATOMIC_RELAXED, AGENT);
        unsigned a = __hip_atomic_fetch_add(bar + grp * 32, 1u, __ATOMIC_RELAXED, AGENT);
        bool released = false;
        if (a == per_group - 1) {
            __hip_atomic_store(bar + grp * 32, 0u, __ATOMIC_RELAXED, AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            unsigned t = __hip_atomic_fetch_add(bar + kBarTop, 1u, __ATOMIC_RELAXED, AGENT);
            if (t == kBarGroups - 1) {
                __hip_atomic_store(bar + kBarTop, 0u, __ATOMIC_RELAXED, AGENT);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __hip_atomic_fetch_add(bar + kBarGen, 1u, __ATOMIC_RELAXED, AGENT);
                released = true;
            }
        }
        if (!released) {
            long spins = 0;
            while (__hip_atomic_load(bar + kBarGen, __ATOMIC_RELAXED, AGENT) == g) {
                if (++spins > kSpinLimit) {
                    __hip_atomic_store(bar + kBarErr, 1u, __ATOMIC_RELAXED, AGENT);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        s_err = __hip_atomic_load(bar + kBarErr, __ATOMIC_RELAXED, AGENT);
    }
    __syncthreads();
    return s_err != 0;
}

// Canonical sum of the lane values `acc` over the grid; every block returns
// the same value.  part: 2 x kRedBlocks doubles, `phase` selects the half.
__device__ __forceinline__ bool grid_sum(double acc, double* part, int phase, unsigned* bar, double* s, double* out) {
    const int tid = threadIdx.x;
    const int lane = tid & (kRedThreads - 1);
    double g = tree256(acc, s);
    double* p = part + phase * kRedBlocks;
    if (lane == 0) __hip_atomic_store(p + blockIdx.x * (kPT / kRedThreads) + tid / kRedThreads, g,
                                      __ATOMIC_RELAXED, AGENT);
    if (grid_sync(bar)) return false;
    // all kRedBlocks partials fetched in parallel (one per thread), then lane t
    // adds partials t, t+256, t+512, t+768 in order and the halving tree finishes
    static_assert(kPT == kRedBlocks, "one partial per thread");
    double pv = __hip_atomic_load(p + tid, __ATOMIC_RELAXED, AGENT);
    s[tid] = pv;
    __syncthreads();
    double a = 0.0;
    if (tid < kRedThreads)
        for (int b = tid; b < kRedBlocks; b += kRedThreads) a = a + s[b];
    __syncthreads();
    double r = tree256(a, s);
    __shared__ double s_out;
    if (tid == 0) s_out = r;
    __syncthreads();
    *out = s_out;
    return true;
}

template <int PER>
__global__ __launch_bounds__(kPT) void k_mgs_resident(const double* wsrc, const double* V, long n, int M, int j,
                                                     double* H, double* vnext, int* ints, double* part,
                                                     unsigned* bar) {
    __shared__ double s[kPT];
    __shared__ int s_stop;
    if (threadIdx.x == 0) s_stop = ints[1];
    __syncthreads();
    if (s_stop) return;
    const long T = (long)kPB * kPT;
    const long t = (long)blockIdx.x * kPT + threadIdx.x;
    // Lanes past the end hold +0.0: their products are +0.0 and adding +0.0
    // to a lane sum that starts at +0.0 leaves it unchanged, so no branch is
    // needed (loads are clamped in range and issued back to back).
    double w[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        long e = t + k * T;
        double x = wsrc[e < n ? e : n - 1];
        w[k] = (e < n) ? x : 0.0;
    }
    __shared__ double s_hcol[kMaxM + 1];
    int phase = 0;
    for (int i = 0; i <= j; ++i) {
        const double* v = V + (long)i * n;
        double vv[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            long e = t + k * T;
            double x = v[e < n ? e : n - 1];
            vv[k] = (e < n) ? x : 0.0;
        }
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < PER; ++k) acc = acc + vv[k] * w[k];
        double h;
        if (!grid_sum(acc, part, phase, bar, s, &h)) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                ints[1] = 1;
                ints[2] |= ROK_FLAG_BARRIER;
            }
            return;
        }
        phase ^= 1;
        if (threadIdx.x == 0) s_hcol[i] = h;
        if (blockIdx.x == 0 && threadIdx.x == 0) H[i * M + j] = h;
#pragma unroll
        for (int k = 0; k < PER; ++k) w[k] = w[k] - h * vv[k];
    }
    if (j + 1 >= M) return;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < PER; ++k) acc = acc + w[k] * w[k];
    double nn;
    if (!grid_sum(acc, part, phase, bar, s, &nn)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ints[1] = 1;
            ints[2] |= ROK_FLAG_BARRIER;
        }
        return;
    }
    const double hn = sqrt(nn);
    double c = 0.0;
    for (int i = 0; i <= j; ++i) c = c + s_hcol[i] * s_hcol[i];
    c = c + hn * hn;
    const bool brk = hn <= kBreakdownTolR * sqrt(c);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        H[(j + 1) * M + j] = hn;
        if (brk) {
            ints[0] = j + 1;
            ints[1] = 1;
            ints[2] |= ROK_FLAG_BREAKDOWN;
        }
        if (!(hn == hn) || hn == __builtin_inf()) ints[2] |= ROK_FLAG_NONFINITE;
    }
    if (brk) return;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        long e = t + k * T;
        if (e < n) vnext[e] = w[k] / hn;
    }
}

template <int PER>
static hipError_t launch_res(const Work& W, const double* w, const double* V, long n, int M, int j, double* vnext,
                             hipStream_t st) {
    long nn = n;
    int MM = M, jj = j;
    double* H = W.H;
    int* ints = W.ints;
    double* part = W.gpart;
    unsigned* bar = W.bar;
    void* args[] = {(void*)&w, (void*)&V, (void*)&nn, (void*)&MM, (void*)&jj, (void*)&H, (void*)&vnext,
                    (void*)&ints, (void*)&part, (void*)&bar};
    return hipLaunchCooperativeKernel((const void*)k_mgs_resident<PER>, dim3(kPB), dim3(kPT), args, 0, st);
}

// Elements per lane the resident kernel supports (0 if n is too large).
int mgs_resident_per(long n) {
    const long T = (long)kPB * kPT;
    long per = (n + T - 1) / T;
    if (per <= 1) return 1;
    if (per <= 2) return 2;
    if (per <= 4) return 4;
    if (per <= 8) return 8;
    if (per <= 16) return 16;
    return 0;
}

static int g_coop_ok = -1;

// True if the device can host the cooperative grid (checked once).
bool mgs_resident_available() {
    if (g_coop_ok >= 0) return g_coop_ok == 1;
    int dev = 0, coop = 0, cus = 0, nb = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_mgs_resident<16>, kPT, 0) != hipSuccess) {
        g_coop_ok = 0;
        return false;
    }
    g_coop_ok = (coop && (long)nb * cus >= kPB) ? 1 : 0;
    return g_coop_ok == 1;
}

hipError_t launch_mgs_resident(const Work& W, const double* w, const double* V, long n, int M, int j, double* vnext,
                               hipStream_t st) {
    switch (mgs_resident_per(n)) {
        case 1: return launch_res<1>(W, w, V, n, M, j, vnext, st);
        case 2: return launch_res<2>(W, w, V, n, M, j, vnext, st);
        case 4: return launch_res<4>(W, w, V, n, M, j, vnext, st);
        case 8: return launch_res<8>(W, w, V, n, M, j, vnext, st);
        case 16: return launch_res<16>(W, w, V, n, M, j, vnext, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rok

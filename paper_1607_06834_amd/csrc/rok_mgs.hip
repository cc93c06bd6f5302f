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
//
// The same machinery runs the reverse of a column for the discrete adjoint
// of the step (k_mgs_rev_resident below): the normalisation and the passes
// in reverse order, with the forward iterate and its adjoint resident.
#include "rok.h"
#include "rok_device.hpp"
#include "rok_kernels.hpp"

namespace rok {

constexpr int kPT = 1024;                       // threads per block
constexpr int kPB = kRedBlocks * kRedThreads / kPT;  // 256 blocks
constexpr double kBreakdownTolR = 1e-13;
constexpr long kSpinLimit = 1L << 22;
// s_waitcnt operand with vmcnt = 0 and the other counters at their maximum
// (gfx9 encoding: vmcnt[3:0] and [15:14], expcnt[6:4], lgkmcnt[11:8]).
constexpr int kWaitVmcnt0 = 0x0F70;

#define AGENT __HIP_MEMORY_SCOPE_AGENT

// Grid barrier, two levels: the blocks are split into kBarGroups groups;
// the last arrival of a group bumps the top counter, the last arrival at the
// top bumps the generation everyone waits on.  Counters sit on separate
// 128-byte lines.  bar (unsigned): [g * 32] group g arrivals, [kBarTop] top
// arrivals, [kBarGen] generation, [kBarErr] error.  Run by thread 0 only;
// returns true if the barrier failed (spin limit).
constexpr int kBarGroups = 16;
constexpr int kBarTop = kBarGroups * 32;
constexpr int kBarGen = kBarTop + 32;
constexpr int kBarErr = kBarGen + 32;

__device__ __forceinline__ bool grid_arrive_wait(unsigned* bar) {
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
    return __hip_atomic_load(bar + kBarErr, __ATOMIC_RELAXED, AGENT) != 0;
}

// Canonical sum of the lane values `acc` over the grid, in two halves so the
// caller can issue independent loads in between: publish() combines the
// block's lanes into its four 256-lane group sums (left in LDS), collect()
// stores them, waits for every block and finishes the sum (every block
// obtains the same bits).  Only wave 0 touches global memory in collect(),
// so the other waves may keep loads in flight across it.
// part: 2 x kRedBlocks doubles, `phase` selects the half.
__device__ __forceinline__ void publish(double acc, double* s, double* gs) {
    const int tid = threadIdx.x;
    const double g = tree256(acc, s);
    if ((tid & (kRedThreads - 1)) == 0) gs[tid / kRedThreads] = g;
}

// Wave 0 stores the block's four partials, runs the barrier and then
// finishes the sum alone: lane l holds the canonical lanes t = l + 64 m
// (m = 0..3), each the in-order sum of partials t, t + 256, t + 512, t + 768;
// the first two levels of the halving tree (t += t + 128, then t += t + 64)
// are additions within the lane and the last six are shuffles, the same
// operations in the same order as the block tree.  after_loads() runs in
// wave 0 once the partial loads are issued (the caller's prefetch: loads
// complete in order, so the sum does not wait for them).
// Returns false (in every thread of the block) if the barrier failed.
template <typename AfterLoads>
__device__ __forceinline__ bool collect(double* part, int phase, unsigned* bar, const double* gs, double* out,
                                        AfterLoads after_loads) {
    const int tid = threadIdx.x;
    __shared__ double s_out;
    __shared__ int s_err;
    static_assert(kPT == kRedBlocks && kRedThreads == 256, "one partial per thread, 256-lane groups");
    __syncthreads();
    if (tid < 64) {
        if (tid < kPT / kRedThreads)
            __hip_atomic_store(part + phase * kRedBlocks + blockIdx.x * (kPT / kRedThreads) + tid, gs[tid],
                               __ATOMIC_RELAXED, AGENT);
        // the partials must have reached the coherent level before the arrival
        __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
        int err = 0;
        if (tid == 0) err = grid_arrive_wait(bar) ? 1 : 0;
        err = __shfl(err, 0, 64);
        if (tid == 0) s_err = err;
        if (!err) {
            const double* p = part + phase * kRedBlocks;
            double pv[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) pv[q] = __hip_atomic_load(p + tid + 64 * q, __ATOMIC_RELAXED, AGENT);
            after_loads();
            double a[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                double x = 0.0;
#pragma unroll
                for (int r = 0; r < 4; ++r) x = x + pv[m + 4 * r];
                a[m] = x;
            }
            a[0] = a[0] + a[2];
            a[1] = a[1] + a[3];
            double v = a[0] + a[1];
#pragma unroll
            for (int h = 32; h > 0; h >>= 1) v = v + __shfl_down(v, h, 64);
            if (tid == 0) s_out = v;
        }
    }
    __syncthreads();
    if (s_err) return false;
    *out = s_out;
    return true;
}

// Buffer descriptor word 3 for raw (untyped, unswizzled) loads on gfx9-class
// devices: data format 32 (a zero format would make every access out of range).
constexpr int kBufWord3 = 0x00020000;

// Sixteenths of the next basis vector the waves 1-15 load before a pass's
// exchange (the rest right after it).  Measured at 1024^2, column time in
// HIP events: all before 105.7 us, half 103.4 us, a quarter 105.1 us, none
// 106.0 us.
constexpr int kPrefetchEarly = 8;

// x[k] = src[t + k T] for the chunks of lane t that lie below n, +0.0 past
// the end.  Raw buffer loads with the range n * 8 bytes: an offset past the
// range reads as zero without touching memory, so the loads need no per-lane
// condition (no exec-masked branches, whose joins would make the compiler
// wait for every outstanding load, prefetches included).  All offsets are in
// the lane's offset register, which is what the range check covers.
// chunks k0 <= k < k1 only (the rest of x untouched)
template <int PER, int K0, int K1, int AUX>
__device__ __forceinline__ void load_chunks(const double* __restrict__ src, long n, int t, double (&x)[PER]) {
    constexpr int T = kPB * kPT;
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(src), (short)0, (int)(n * 8), kBufWord3);
    int off = t * 8;
    asm volatile("" : "+v"(off));
#pragma unroll
    for (int k = K0; k < K1; ++k)
        x[k] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off + k * T * 8, 0, AUX));
}

template <int PER, int AUX = 0>
__device__ __forceinline__ void load_lane(const double* __restrict__ src, long n, int t, double (&x)[PER]) {
    constexpr int T = kPB * kPT;
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(src), (short)0, (int)(n * 8), kBufWord3);
    // an opaque base offset: the chunk offsets are formed next to each load
    // instead of being held in registers across the whole kernel
    int off = t * 8;
    asm volatile("" : "+v"(off));
#pragma unroll
    for (int k = 0; k < PER; ++k)
        x[k] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off + k * T * 8, 0, AUX));
}

// dst[t + k T] = x[k] for the chunks of lane t below n (raw buffer stores
// with the range n * 8 bytes: stores past it are dropped).
template <int PER>
__device__ __forceinline__ void store_lane(double* __restrict__ dst, long n, int t, const double (&x)[PER]) {
    constexpr int T = kPB * kPT;
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(dst, (short)0, (int)(n * 8), kBufWord3);
    using B64 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    int off = t * 8;
    asm volatile("" : "+v"(off));
#pragma unroll
    for (int k = 0; k < PER; ++k)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(B64, x[k]), r, off + k * T * 8, 0, 0);
}

// Work vector storage of one lane: registers, or (PER = 16, where three
// register arrays of 16 doubles would exceed the 128 registers a lane has at
// 1024 threads per block) the lane's own LDS slots, used as private storage.
template <int PER, bool LDSW>
struct LaneVec {
    double r[LDSW ? 1 : PER];
    double* l;
    __device__ __forceinline__ double get(int k) const { return LDSW ? l[k * kPT + threadIdx.x] : r[k]; }
    __device__ __forceinline__ void set(int k, double x) {
        if constexpr (LDSW) l[k * kPT + threadIdx.x] = x;
        else r[k] = x;
    }
};

template <int PER>
__global__ __launch_bounds__(kPT) void k_mgs_resident(const double* wsrc, const double* V, long n, int M, int j,
                                                     double* H, double* vnext, int* ints, double* part,
                                                     unsigned* bar) {
    constexpr bool LDSW = PER >= 16;
    __shared__ double s[kPT];
    __shared__ double s_w[LDSW ? PER * kPT : 1];
    __shared__ int s_stop;
    if (threadIdx.x == 0) s_stop = ints[1];
    __syncthreads();
    if (s_stop) return;
    constexpr long T = (long)kPB * kPT;
    const int t = blockIdx.x * kPT + threadIdx.x;
    const int nk = (t < n) ? (int)((n - 1 - t) / T) + 1 : 0;   // chunks of lane t inside the vector
    // Wave 0 runs the grid barrier; the other waves issue the loads of the
    // next basis vector as soon as its register array is free (right after
    // the pass's update), so they stay in flight across the block tree and
    // the exchange, and wave 0 issues its own behind the loads of the
    // partials.  A pass then costs about max(load, tree + exchange).  Two
    // basis-vector arrays alternate: at pass i one holds v_{i-1} (for the
    // update w -= h v_{i-1}) and v_{i+1} is loaded into it after use.
    const bool prefetch = threadIdx.x >= 64;
    // Lanes past the end hold +0.0: their products are +0.0 and adding +0.0
    // to a lane sum that starts at +0.0 leaves it unchanged.
    LaneVec<PER, LDSW> w;
    w.l = s_w;
    {
        double x[PER];
        load_lane<PER>(wsrc, n, t, x);
#pragma unroll
        for (int k = 0; k < PER; ++k) w.set(k, x[k]);
    }
    double A[PER], B[PER];
    load_lane<PER, 2>(V, n, t, A);
    __shared__ double s_hcol[kMaxM + 1];
    __shared__ double s_gs[kPT / kRedThreads];
    int phase = 0;
    double h = 0.0;
    bool failed = false;
    auto none = [] {};
    // Pass i with cur = v_i and prev = v_{i-1}: w -= h_{i-1} prev (i > 0),
    // h_i = <v_i, w>, then prev <- v_{i+1}.
    auto pass = [&](int i, double (&cur)[PER], double (&prev)[PER]) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            double wk = w.get(k);
            if (i > 0) {
                wk = wk - h * prev[k];
                w.set(k, wk);
            }
            acc = acc + cur[k] * wk;
        }
        // the sum is complete before the loads are issued: otherwise the
        // products sink past the (conditional) loads and the merge after them
        // waits for every outstanding load, the prefetch included
        asm volatile("" : "+v"(acc) : : "memory");
        const bool more = i < j;
        // waves 1-15: the first kPrefetchEarly sixteenths of v_{i+1} before the exchange, the
        // rest after it (the exchange's loads queue behind whatever stream is in flight)
        constexpr int KS = (PER * kPrefetchEarly) / 16;
        if (more && prefetch) load_chunks<PER, 0, KS, 2>(V + (long)(i + 1) * n, n, t, prev);
        publish(acc, s, s_gs);
        // unconditional (v_j again after the last pass, 64 lanes' worth), so
        // that the sum's waits count exactly these loads behind the partials
        auto wave0_prefetch = [&] { load_lane<PER, 2>(V + (long)(more ? i + 1 : j) * n, n, t, prev); };
        if (!collect(part, phase, bar, s_gs, &h, wave0_prefetch)) {
            failed = true;
            return;
        }
        phase ^= 1;
        if (more && prefetch) load_chunks<PER, KS, PER, 2>(V + (long)(i + 1) * n, n, t, prev);
        if (threadIdx.x == 0) s_hcol[i] = h;
        if (blockIdx.x == 0 && threadIdx.x == 0) H[i * M + j] = h;
    };
    int i = 0;
    for (;;) {
        pass(i, A, B);
        if (failed || i == j) break;
        ++i;
        pass(i, B, A);
        if (failed || i == j) break;
        ++i;
    }
    if (failed) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ints[1] = 1;
            ints[2] |= ROK_FLAG_BARRIER;
        }
        return;
    }
    // last update w -= h_j v_j (v_j is A after an even number of passes, else B)
    const bool inA = (j % 2) == 0;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const double wk = w.get(k) - h * (inA ? A[k] : B[k]);
        w.set(k, wk);
        acc = acc + wk * wk;
    }
    if (j + 1 >= M) return;
    publish(acc, s, s_gs);
    double nn;
    if (!collect(part, phase, bar, s_gs, &nn, none)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ints[1] = 1;
            ints[2] |= ROK_FLAG_BARRIER;
        }
        return;
    }
    const double hn = sqrt(nn);
    double c = 0.0;
    for (int q = 0; q <= j; ++q) c = c + s_hcol[q] * s_hcol[q];
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
    for (int k = 0; k < PER; ++k)
        if (k < nk) vnext[t + k * T] = w.get(k) / hn;
}

// Reverse of one Arnoldi column (the discrete adjoint of its modified
// Gram-Schmidt passes and of the normalisation v_{j+1} = w / h_{j+1,j}),
// resident like the forward kernel: w (the forward iterates, rebuilt pass
// by pass) and wbar stay in registers, so reverse pass i streams only
// v_{i-1} (for the next dot) and reads and writes vbar_i.  Rules, with x'
// the result of a forward operation:
//   v = w / rho, rho = ||w||:  wbar = vbar / rho + (Hbar_rho - <vbar, v> / rho) v
//   w' = w - h v, h = <v, w>:  hb = Hbar_h - <w'bar, v>, w = w' + h v,
//                              vbar += hb w - h w'bar, wbar = w'bar + hb v
// The final forward iterate is h_{j+1,j} v_{j+1} where v_{j+1} exists, else
// (the basis' last column) J v_j - sum_i h_ij v_i with J v_j read from wsrc.
// Every dot product is the canonical sum (the same lane order and finish as
// the per-pass reverse kernels, whose results this reproduces bit for bit).
// Nothing runs for j >= M_eff or after a failed in-kernel barrier.
template <int PER>
__global__ __launch_bounds__(kPT) void k_mgs_rev_resident(const double* wsrc, const double* V, double* Vbar,
                                                         const double* H, const double* Hbar, long n, int M, int j,
                                                         double* wbar_out, int* ints, double* part, unsigned* bar) {
    __shared__ double s[kPT];
    __shared__ double s_gs[kPT / kRedThreads];
    __shared__ int s_m, s_bad;
    __shared__ double s_h[kMaxM + 1], s_hb[kMaxM + 1];   // column j of H and Hbar
    if (threadIdx.x == 0) {
        s_m = ints[0];
        s_bad = (ints[2] & ROK_FLAG_BARRIER) != 0;
    }
    if (threadIdx.x < M && threadIdx.x <= j + 1) {
        s_h[threadIdx.x] = H[threadIdx.x * M + j];
        s_hb[threadIdx.x] = Hbar[threadIdx.x * M + j];
    }
    __syncthreads();
    const int m = s_m;
    if (j >= m || s_bad) return;
    const int t = blockIdx.x * kPT + threadIdx.x;
    const bool prefetch = threadIdx.x >= 64;
    const bool nrm = j + 1 < m;
    double w[PER], wb[PER], A[PER], B[PER], vb[PER];
    int phase = 0;
    double d = 0.0;
    bool failed = false;
    // canonical sum of the lane values acc; loads(): the caller's prefetch,
    // issued by waves 1.. before the block tree and by wave 0 behind the partials
    auto exchange = [&](double acc, auto loads) {
        asm volatile("" : "+v"(acc) : : "memory");
        if (prefetch) loads();
        publish(acc, s, s_gs);
        if (!collect(part, phase, bar, s_gs, &d, loads)) failed = true;
        phase ^= 1;
    };
    if (nrm) {
        load_lane<PER>(V + (long)(j + 1) * n, n, t, A);      // v_{j+1}
        load_lane<PER>(Vbar + (long)(j + 1) * n, n, t, vb);  // vbar_{j+1}
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < PER; ++k) acc = acc + vb[k] * A[k];
        exchange(acc, [&] { load_lane<PER>(V + (long)j * n, n, t, B); });
        if (failed) goto fail;
        const double rho = s_h[j + 1];
        const double coef = s_hb[j + 1] - d / rho;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            w[k] = rho * A[k];
            wb[k] = vb[k] / rho + coef * A[k];
        }
    } else {
        load_lane<PER>(wsrc, n, t, w);
        for (int i = 0; i <= j; ++i) {
            load_lane<PER>(V + (long)i * n, n, t, B);
            const double hij = s_h[i];
#pragma unroll
            for (int k = 0; k < PER; ++k) w[k] = w[k] - hij * B[k];
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) wb[k] = 0.0;
    }
    {   // <wbar, v_j>; meanwhile v_{j-1} and vbar_j arrive
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < PER; ++k) acc = acc + wb[k] * B[k];
        exchange(acc, [&] {
            load_lane<PER>(V + (long)(j > 0 ? j - 1 : 0) * n, n, t, A);
            load_lane<PER>(Vbar + (long)j * n, n, t, vb);
        });
        if (failed) goto fail;
    }
    {
        // reverse pass i with cur = v_i, prev = v_{i-1}, vb = vbar_i, d = <wbar, v_i>
        auto rpass = [&](int i, double (&cur)[PER], double (&prev)[PER]) {
            const double h = s_h[i];
            const double hb = s_hb[i] - d;
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                const double v = cur[k];
                const double wo = w[k] + h * v;
                w[k] = wo;
                const double b = wb[k];
                vb[k] = vb[k] + hb * wo - h * b;
                const double wn = b + hb * v;
                wb[k] = wn;
                acc = acc + wn * prev[k];
            }
            store_lane<PER>(Vbar + (long)i * n, n, t, vb);
            if (i == 0) return;
            exchange(acc, [&] {
                load_lane<PER>(V + (long)(i > 1 ? i - 2 : 0) * n, n, t, cur);
                load_lane<PER>(Vbar + (long)(i - 1) * n, n, t, vb);
            });
        };
        int i = j;
        for (;;) {
            rpass(i, B, A);
            if (failed || i == 0) break;
            --i;
            rpass(i, A, B);
            if (failed || i == 0) break;
            --i;
        }
        if (failed) goto fail;
    }
    store_lane<PER>(wbar_out, n, t, wb);
    return;
fail:
    if (blockIdx.x == 0 && threadIdx.x == 0) ints[2] |= ROK_FLAG_BARRIER;
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

template <int PER>
static hipError_t launch_rev(const Work& W, const AdjWork& A, long n, int M, int j, hipStream_t st) {
    long nn = n;
    int MM = M, jj = j;
    const double* wsrc = W.w;
    const double* V = W.V;
    double* Vbar = A.Vbar;
    const double* H = W.H;
    const double* Hbar = A.Hbar;
    double* wbar = A.wbar;
    int* ints = W.ints;
    double* part = W.gpart;
    unsigned* bar = W.bar;
    void* args[] = {(void*)&wsrc, (void*)&V,  (void*)&Vbar, (void*)&H,    (void*)&Hbar, (void*)&nn,
                    (void*)&MM,   (void*)&jj, (void*)&wbar, (void*)&ints, (void*)&part, (void*)&bar};
    return hipLaunchCooperativeKernel((const void*)k_mgs_rev_resident<PER>, dim3(kPB), dim3(kPT), args, 0, st);
}

static int g_rev_ok = -1;

// The resident reverse keeps five lane vectors in registers: up to 8 elements per lane.
bool mgs_rev_resident_available(long n) {
    const int per = mgs_resident_per(n);
    if (per == 0 || per > 8) return false;
    if (g_rev_ok < 0) {
        int dev = 0, coop = 0, cus = 0, nb = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)k_mgs_rev_resident<8>, kPT, 0) != hipSuccess)
            g_rev_ok = 0;
        else
            g_rev_ok = (coop && (long)nb * cus >= kPB) ? 1 : 0;
    }
    return g_rev_ok == 1;
}

hipError_t launch_mgs_rev_resident(const Work& W, const AdjWork& A, int M, int j, long n, hipStream_t st) {
    switch (mgs_resident_per(n)) {
        case 1: return launch_rev<1>(W, A, n, M, j, st);
        case 2: return launch_rev<2>(W, A, n, M, j, st);
        case 4: return launch_rev<4>(W, A, n, M, j, st);
        case 8: return launch_rev<8>(W, A, n, M, j, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rok

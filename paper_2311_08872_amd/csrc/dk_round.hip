// dk_round.hip -- the persistent round kernel: every resident level of one Algorithm-1 round
// (Sec. 7) in a single launch.
//
// The host cuts the round into tasks (a level and a contiguous range of its sample indices),
// ordered by decreasing cost per sample (finest pair first), and uploads the task list.  A grid of
// one 1024-lane block per compute unit then pulls task indices from a device counter: a block
// takes the next index, runs the task's samples in block-iterations of SPW samples with the same
// level_body as the per-level kernel (8 rows per lane at every grid size; 1024 lanes hold 256
// samples of 8 x 8, 64 of 16 x 16, 16 of 32 x 32, 4 of 64 x 64 or one 128 x 128 sample), and
// folds the per-sample values into the task's compensated moment sums in sample order.  The host
// merges the task sums of each level in task order, so the result depends on the task list only,
// not on which block ran which task or when.  Every block leaves the loop once the counter passes
// the number of tasks.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dk_round.h"
#include "dk_level.h"

namespace dk {

namespace {
constexpr int RT = 1024;     // lanes per block
constexpr int RR = 8;        // rows per lane
constexpr int RC = 2;        // columns per lane

template <int NF>
constexpr int round_spw() { return RT / ((NF / RC) * (NF / RR)); }

template <int NF, bool PAIR>
constexpr int round_lds() { return round_spw<NF>() * halo_elems<NF, RR, PAIR>(); }

constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int RHALO = cmax(cmax(cmax(round_lds<8, false>(), round_lds<16, false>()),
                                cmax(round_lds<32, false>(), round_lds<64, false>())),
                           cmax(cmax(round_lds<128, false>(), round_lds<16, true>()),
                                cmax(cmax(round_lds<32, true>(), round_lds<64, true>()), round_lds<128, true>())));
static_assert(RHALO * 4 <= 96 * 1024, "round kernel LDS");

// The lane index is passed through an empty asm statement so that the compiler cannot hoist the
// lane constants of all nine level kinds out of the task loop (they would all stay live at once).
template <int NF, bool PAIR, int FLUX>
__device__ __forceinline__ void body(const LevelArgs& A, float* halo, double* red)
{
    int tid = (int)threadIdx.x;
    asm volatile("" : "+v"(tid));
    __builtin_assume(tid >= 0 && tid < RT);
    level_body<float, NF, RR, RC, PAIR, FLUX, true, round_spw<NF>()>(A, 0, halo, red, tid);
}
}  // namespace

// level kinds of the round kernel: singles 8..128 are 0..4, pairs 16..128 are 5..8; -1 = none
int round_kind(int nf, bool pair)
{
    switch (nf) {
        case 8: return pair ? -1 : 0;
        case 16: return pair ? 5 : 1;
        case 32: return pair ? 6 : 2;
        case 64: return pair ? 7 : 3;
        case 128: return pair ? 8 : 4;
        default: return -1;
    }
}

int round_spw_of(int nf)
{
    switch (nf) {
        case 8: return round_spw<8>();
        case 16: return round_spw<16>();
        case 32: return round_spw<32>();
        case 64: return round_spw<64>();
        case 128: return round_spw<128>();
        default: return 0;
    }
}

__global__ void round_reset_kernel(uint32_t* head)
{
    if (threadIdx.x == 0) *head = 0u;
}

template <int FLUX>
__global__ void __launch_bounds__(RT) round_kernel(const RoundArgs P)
{
    __shared__ float halo[RHALO];
    __shared__ double red[RT / 64];
    __shared__ uint32_t s_task;
    const int tid = threadIdx.x;
    const int nobs = P.n_obs;
    const int nmom = nobs * DK_NMOM;
    double* scr = P.scratch + (size_t)blockIdx.x * P.scratch_stride;
    const uint32_t ntasks = *P.ntasks;
    for (;;) {
        if (tid == 0) s_task = atomicAdd(P.head, 1u);
        __syncthreads();
        const uint32_t t = __builtin_amdgcn_readfirstlane(s_task);
        __syncthreads();
        if (t >= ntasks) break;
        const RoundTask task = P.tasks[t];
        const RoundLevel& L = P.levels[task.level];
        const int kind = L.kind;
        const uint64_t spw = (uint64_t)L.spw;
        double* tm = P.task_mom + (size_t)t * nmom * 2;
        for (uint64_t it = 0; it < task.count; it += spw) {
            LevelArgs A = L.A;
            A.first = task.first + it;
            A.count = task.count - it < spw ? task.count - it : spw;
            A.out = scr;
            A.field_f = nullptr;
            A.field_c = nullptr;
            switch (kind) {
                case 0: body<8, false, FLUX>(A, halo, red); break;
                case 1: body<16, false, FLUX>(A, halo, red); break;
                case 2: body<32, false, FLUX>(A, halo, red); break;
                case 3: body<64, false, FLUX>(A, halo, red); break;
                case 4: body<128, false, FLUX>(A, halo, red); break;
                case 5: body<16, true, FLUX>(A, halo, red); break;
                case 6: body<32, true, FLUX>(A, halo, red); break;
                case 7: body<64, true, FLUX>(A, halo, red); break;
                case 8: body<128, true, FLUX>(A, halo, red); break;
                default: break;   // no such kind: the host never lists one
            }
            __syncthreads();
            // lane (j, k) folds moment k of observable j over this iteration's samples, in order
            if (tid < nmom) {
                const int j = tid / DK_NMOM, k = tid % DK_NMOM;
                double s = 0.0, c = 0.0;
                if (it > 0) { s = tm[2 * tid]; c = tm[2 * tid + 1]; }
                for (uint64_t i = 0; i < A.count; ++i) {
                    const double pf = scr[(i * nobs + j) * 2 + 0];
                    const double pc = scr[(i * nobs + j) * 2 + 1];
                    const double y = pf - pc;
                    double v;
                    switch (k) {
                        case DK_MOM_Y: v = y; break;
                        case DK_MOM_Y2: v = y * y; break;
                        case DK_MOM_PF: v = pf; break;
                        case DK_MOM_PF2: v = pf * pf; break;
                        case DK_MOM_PC: v = pc; break;
                        default: v = pc * pc; break;
                    }
                    neumaier(s, c, v);
                }
                tm[2 * tid] = s;
                tm[2 * tid + 1] = c;
            }
            __syncthreads();
        }
    }
}

int round_blocks_per_cu(int flux)
{
    int nb = 0;
    const hipError_t e = flux == DK_FLUX_STAGGERED
                             ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, round_kernel<DK_FLUX_STAGGERED>, RT, 0)
                             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, round_kernel<DK_FLUX_CENTRAL>, RT, 0);
    return e == hipSuccess && nb > 0 ? nb : 1;
}

int round_max_obs() { return RT / DK_NMOM; }

hipError_t launch_round(const RoundArgs& P, int flux, int grid, hipStream_t s)
{
    if (grid <= 0 || P.n_obs <= 0 || P.n_obs * DK_NMOM > RT) return hipErrorInvalidValue;
    hipLaunchKernelGGL(round_reset_kernel, dim3(1), dim3(64), 0, s, P.head);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (flux == DK_FLUX_STAGGERED)
        hipLaunchKernelGGL(round_kernel<DK_FLUX_STAGGERED>, dim3(grid), dim3(RT), 0, s, P);
    else
        hipLaunchKernelGGL(round_kernel<DK_FLUX_CENTRAL>, dim3(grid), dim3(RT), 0, s, P);
    return hipGetLastError();
}

}  // namespace dk

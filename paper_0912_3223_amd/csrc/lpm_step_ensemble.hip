// Ensemble launches of the persistent step kernel with LPM_SLICE_BLOCK
// threads per block: two or three wind components, steady or hourly fields,
// uniform levels, one or two nuclides, K_z kinds 0-2, deposition on/off.
// The build compiles this file once per block size (128, 256, 512), so the
// block sizes the autotuner chooses from compile in parallel.
#include "lpm_host.h"
#include "lpm_step.h"

#ifndef LPM_SLICE_BLOCK
#error "compile with -DLPM_SLICE_BLOCK=128|256|512"
#endif

namespace lpm_host {
namespace {

// Launches the variant on `grid` resident blocks, or with `plan` only
// stores that block count (nothing is launched).
template <int BLOCK, int NCOMP, bool TIME, int NNUC, int KZ, bool DEP>
void go(unsigned nb, hipStream_t s, const lpm::StepConst& p, int bpc, unsigned* plan)
{
    auto k = lpm::step_kernel<BLOCK, NCOMP, TIME, false, NNUC, KZ, DEP, true>;
    const unsigned grid = resident_blocks(reinterpret_cast<const void*>(k), BLOCK, bpc, nb);
    if (plan) *plan = grid;
    else hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, s, p);
}

template <int BLOCK, int NCOMP, bool TIME, int NNUC>
void by_kz(int kz, bool dep, unsigned nb, hipStream_t s, const lpm::StepConst& p, int bpc,
           unsigned* plan)
{
    switch (kz) {
    case 0: dep ? go<BLOCK, NCOMP, TIME, NNUC, 0, true>(nb, s, p, bpc, plan)
                : go<BLOCK, NCOMP, TIME, NNUC, 0, false>(nb, s, p, bpc, plan); break;
    case 1: dep ? go<BLOCK, NCOMP, TIME, NNUC, 1, true>(nb, s, p, bpc, plan)
                : go<BLOCK, NCOMP, TIME, NNUC, 1, false>(nb, s, p, bpc, plan); break;
    default: dep ? go<BLOCK, NCOMP, TIME, NNUC, 2, true>(nb, s, p, bpc, plan)
                 : go<BLOCK, NCOMP, TIME, NNUC, 2, false>(nb, s, p, bpc, plan); break;
    }
}

template <int BLOCK, int NCOMP, bool TIME>
void by_nnuc(int nnuc, int kz, bool dep, unsigned nb, hipStream_t s, const lpm::StepConst& p,
             int bpc, unsigned* plan)
{
    if (nnuc == 1) by_kz<BLOCK, NCOMP, TIME, 1>(kz, dep, nb, s, p, bpc, plan);
    else by_kz<BLOCK, NCOMP, TIME, 2>(kz, dep, nb, s, p, bpc, plan);
}

}  // namespace

template <int BLOCK>
void launch_ensemble(int ncomp, bool time, int nnuc, int kz, bool dep, unsigned nb, hipStream_t s,
                     const lpm::StepConst& p, int blocks_per_cu, unsigned* plan)
{
    if (ncomp == 2) {
        if (time) by_nnuc<BLOCK, 2, true>(nnuc, kz, dep, nb, s, p, blocks_per_cu, plan);
        else by_nnuc<BLOCK, 2, false>(nnuc, kz, dep, nb, s, p, blocks_per_cu, plan);
    } else {
        if (time) by_nnuc<BLOCK, 3, true>(nnuc, kz, dep, nb, s, p, blocks_per_cu, plan);
        else by_nnuc<BLOCK, 3, false>(nnuc, kz, dep, nb, s, p, blocks_per_cu, plan);
    }
}

template void launch_ensemble<LPM_SLICE_BLOCK>(int, bool, int, int, bool, unsigned, hipStream_t,
                                               const lpm::StepConst&, int, unsigned*);

}  // namespace lpm_host

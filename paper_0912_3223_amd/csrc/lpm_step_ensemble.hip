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

template <int BLOCK, int NCOMP, bool TIME, int NNUC, int KZ, bool DEP>
void go(unsigned nb, hipStream_t s, const lpm::StepConst& p, int bpc)
{
    auto k = lpm::step_kernel<BLOCK, NCOMP, TIME, false, NNUC, KZ, DEP, true>;
    const unsigned grid = resident_blocks(reinterpret_cast<const void*>(k), BLOCK, bpc, nb);
    hipLaunchKernelGGL(k, dim3(grid), dim3(BLOCK), 0, s, p);
}

template <int BLOCK, int NCOMP, bool TIME, int NNUC>
void by_kz(int kz, bool dep, unsigned nb, hipStream_t s, const lpm::StepConst& p, int bpc)
{
    switch (kz) {
    case 0: dep ? go<BLOCK, NCOMP, TIME, NNUC, 0, true>(nb, s, p, bpc)
                : go<BLOCK, NCOMP, TIME, NNUC, 0, false>(nb, s, p, bpc); break;
    case 1: dep ? go<BLOCK, NCOMP, TIME, NNUC, 1, true>(nb, s, p, bpc)
                : go<BLOCK, NCOMP, TIME, NNUC, 1, false>(nb, s, p, bpc); break;
    default: dep ? go<BLOCK, NCOMP, TIME, NNUC, 2, true>(nb, s, p, bpc)
                 : go<BLOCK, NCOMP, TIME, NNUC, 2, false>(nb, s, p, bpc); break;
    }
}

template <int BLOCK, int NCOMP, bool TIME>
void by_nnuc(int nnuc, int kz, bool dep, unsigned nb, hipStream_t s, const lpm::StepConst& p,
             int bpc)
{
    if (nnuc == 1) by_kz<BLOCK, NCOMP, TIME, 1>(kz, dep, nb, s, p, bpc);
    else by_kz<BLOCK, NCOMP, TIME, 2>(kz, dep, nb, s, p, bpc);
}

}  // namespace

template <int BLOCK>
void launch_ensemble(int ncomp, bool time, int nnuc, int kz, bool dep, unsigned nb, hipStream_t s,
                     const lpm::StepConst& p, int blocks_per_cu)
{
    if (ncomp == 2) {
        if (time) by_nnuc<BLOCK, 2, true>(nnuc, kz, dep, nb, s, p, blocks_per_cu);
        else by_nnuc<BLOCK, 2, false>(nnuc, kz, dep, nb, s, p, blocks_per_cu);
    } else {
        if (time) by_nnuc<BLOCK, 3, true>(nnuc, kz, dep, nb, s, p, blocks_per_cu);
        else by_nnuc<BLOCK, 3, false>(nnuc, kz, dep, nb, s, p, blocks_per_cu);
    }
}

template void launch_ensemble<LPM_SLICE_BLOCK>(int, bool, int, int, bool, unsigned, hipStream_t,
                                               const lpm::StepConst&, int);

}  // namespace lpm_host

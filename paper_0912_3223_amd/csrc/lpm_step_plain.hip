// Plain (single-release) launches of the persistent step kernel for one
// slice of its compile-time variants: LPM_SLICE_NCOMP wind components and
// steady (LPM_SLICE_TIME = 0), time-interpolated (1) or time-pair-copy (2)
// fields, with every level, nuclide-count, K_z and deposition variant of
// that slice.  The build compiles this file once per slice, so the slices
// compile in parallel.
#include "lpm_host.h"
#include "lpm_step.h"

#if !defined(LPM_SLICE_NCOMP) || !defined(LPM_SLICE_TIME)
#error "compile with -DLPM_SLICE_NCOMP=2|3 -DLPM_SLICE_TIME=0|1|2"
#endif

namespace lpm_host {
namespace {

template <int NCOMP, int TIME, bool LEV, int NNUC, int KZ, bool DEP>
void go(unsigned nb, hipStream_t s, const lpm::StepConst& p, int bpc)
{
    auto k = lpm::step_kernel<lpm::kBlock, NCOMP, TIME, LEV, NNUC, KZ, DEP, false>;
    const unsigned grid = resident_blocks(reinterpret_cast<const void*>(k), lpm::kBlock, bpc, nb);
    hipLaunchKernelGGL(k, dim3(grid), dim3(lpm::kBlock), 0, s, p);
}

template <int NCOMP, int TIME, bool LEV, int NNUC>
void by_kz(int kz, bool dep, unsigned nb, hipStream_t s, const lpm::StepConst& p, int bpc)
{
    switch (kz) {
    case 0: dep ? go<NCOMP, TIME, LEV, NNUC, 0, true>(nb, s, p, bpc)
                : go<NCOMP, TIME, LEV, NNUC, 0, false>(nb, s, p, bpc); break;
    case 1: dep ? go<NCOMP, TIME, LEV, NNUC, 1, true>(nb, s, p, bpc)
                : go<NCOMP, TIME, LEV, NNUC, 1, false>(nb, s, p, bpc); break;
    case 2: dep ? go<NCOMP, TIME, LEV, NNUC, 2, true>(nb, s, p, bpc)
                : go<NCOMP, TIME, LEV, NNUC, 2, false>(nb, s, p, bpc); break;
    // general kernel (Eq. 3 with stability, chains, stochastic deposition)
    default: go<NCOMP, TIME, LEV, NNUC, 4, true>(nb, s, p, bpc); break;
    }
}

template <int NCOMP, int TIME, bool LEV>
void by_nnuc(int nnuc, int kz, bool dep, unsigned nb, hipStream_t s, const lpm::StepConst& p,
             int bpc)
{
    switch (nnuc) {
    case 1: by_kz<NCOMP, TIME, LEV, 1>(kz, dep, nb, s, p, bpc); break;
    case 2: by_kz<NCOMP, TIME, LEV, 2>(kz, dep, nb, s, p, bpc); break;
    case 3: by_kz<NCOMP, TIME, LEV, 3>(kz, dep, nb, s, p, bpc); break;
    default: by_kz<NCOMP, TIME, LEV, 4>(kz, dep, nb, s, p, bpc); break;
    }
}

}  // namespace

template <int NCOMP, int TIME>
void launch_plain(bool lev, int nnuc, int kz, bool dep, unsigned nb, hipStream_t s,
                  const lpm::StepConst& p, int blocks_per_cu)
{
    if (lev) by_nnuc<NCOMP, TIME, true>(nnuc, kz, dep, nb, s, p, blocks_per_cu);
    else by_nnuc<NCOMP, TIME, false>(nnuc, kz, dep, nb, s, p, blocks_per_cu);
}

template void launch_plain<LPM_SLICE_NCOMP, LPM_SLICE_TIME>(
    bool, int, int, bool, unsigned, hipStream_t, const lpm::StepConst&, int);

}  // namespace lpm_host

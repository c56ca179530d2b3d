// Host-side helpers shared by the translation units of liblpm: error
// reporting, argument checks, device attributes, the folding of the C-ABI
// structs into the per-launch constants of the step kernels, and the launch
// dispatch of the step-kernel variants (instantiated in their own units).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lpm.h"
#include "lpm_device.h"

namespace lpm_host {

constexpr int kMsgLen = 512;
extern thread_local char g_msg[kMsgLen];  // message of the last failed call

int fail(int code, const char* fmt, ...);  // sets g_msg, returns code
int hip_status(const char* what);          // LPM_EHIP if a launch failed
bool aligned4(const void* p);
long long first_local_born_at_or_after(const lpm_schedule* sch, long long s);
int check_physics(const lpm_physics* ph);
int check_grid(const lpm_grid* g, bool two_d);
double a0_of(const lpm_source* src, const lpm_schedule* sch, const lpm_physics* ph);
unsigned blocks_for(long long n);
int fill_field(lpm::StepConst& p, const lpm_field* f);
void fill_source(lpm::StepConst& p, const lpm_source* src, const lpm_schedule* sch,
                 const lpm_physics* ph);
void fill_physics(lpm::StepConst& p, const lpm_physics* ph);
int check_field_steps(const lpm::StepConst& p, const lpm_field* f, long long step0,
                      long long n_steps);
void fill_depgrid(lpm::StepConst& p, const lpm_grid& dg);
void activity_coefficients(const lpm_physics* ph, double bc[4][4]);

// Attributes of the current device, read once per device: compute units and
// the most LDS one block may use (bytes).
int device_cus();
int device_lds();

// Blocks of one persistent launch of `kernel` with `block` threads: at most
// what the device holds at once (occupancy cached per kernel and device), at
// most blocks_per_cu per compute unit when that is positive, and at most
// `wanted`.
unsigned resident_blocks(const void* kernel, int block, int blocks_per_cu, unsigned wanted);

// Launch settings of plain step launches (lpm_set_launch).
lpm_launch plain_launch();

// Plain step launch of the variant (NCOMP wind components, time-interpolated
// fields or not, nonuniform levels, nuclide count, K_z kind -- 4 = the
// general kernel -- and deposition on/off); defined, one slice of NCOMP x
// TIME per unit, in lpm_step_plain.hip.
template <int NCOMP, int TIME>
void launch_plain(bool lev, int nnuc, int kz, bool dep, unsigned nb, hipStream_t s,
                  const lpm::StepConst& p, int blocks_per_cu);

// Ensemble step launch with `block` threads per block (128, 256 or 512);
// defined, one block size per unit, in lpm_step_ensemble.hip.  With `plan`
// nothing is launched: *plan receives the number of blocks the launch
// would take.
template <int BLOCK>
void launch_ensemble(int ncomp, bool time, int nnuc, int kz, bool dep, unsigned nb,
                     hipStream_t s, const lpm::StepConst& p, int blocks_per_cu,
                     unsigned* plan = nullptr);

}  // namespace lpm_host

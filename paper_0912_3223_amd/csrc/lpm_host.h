// Host-side helpers shared by the translation units of liblpm: error
// reporting, argument checks and the folding of the C-ABI structs into the
// per-launch constants of the step kernels.
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
double a0_of(const lpm_source* src, const lpm_schedule* sch, const lpm_physics* ph);
unsigned blocks_for(long long n);
int fill_field(lpm::StepConst& p, const lpm_field* f);
void fill_source(lpm::StepConst& p, const lpm_source* src, const lpm_schedule* sch,
                 const lpm_physics* ph);
void fill_physics(lpm::StepConst& p, const lpm_physics* ph);
void activity_coefficients(const lpm_physics* ph, double bc[4][4]);

}  // namespace lpm_host

// Library-internal services shared by the plan code (capi.cpp) and the request server
// (server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "cavity.h"
#include "kernels.hpp"

namespace cav {

// Device blocks from the process-wide cache of the library (hipMalloc only on a miss).
// release: the caller guarantees that no queued work still uses the block.
int device_block_acquire(size_t bytes, void** out);
void device_block_release(void* ptr, size_t bytes);

// Record the status and message of the calling thread's last error (cavity_last_error).
int record_error(int status, const char* msg);

// Whether a caller's device array of complex values meets the 16-byte alignment the
// kernels' complex accesses assume (a null pointer passes).
inline bool aligned16(const void* p) { return (reinterpret_cast<size_t>(p) & 15) == 0; }

// What the RCS of stored solutions needs from a plan: its sizes, the padded solutions
// (nsol of them, nvec entries each), its stream and device, and the number of blocks per
// query of the aperture-transform reduction.
struct PlanView {
  Geo g;
  const zd* xsol;
  long long nvec;
  int nsol;
  hipStream_t stream;
  int device;
  int rcs_blocks;
};
int plan_view(cavity_plan plan, PlanView* out);

// Device bytes one more right-hand side of a lockstep group adds to a plan with these
// arguments (Krylov and transform workspace, solution, gathered column data of a group).
int footprint_per_rhs(double a, double b, double c, int Nx, int Ny, int Nz, const cavity_eps* eps,
                      double k, const cavity_opts* opts, size_t* bytes);

// Move a plan to stream st: all its later work is queued there.  The caller guarantees
// that no work of the plan is pending on its previous stream.
int plan_set_stream(cavity_plan plan, hipStream_t st);

}  // namespace cav

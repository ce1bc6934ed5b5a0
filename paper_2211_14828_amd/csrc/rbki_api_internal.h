// Entry points shared between the C ABI (api.hip) and the request server
// (serve.hip).  Internal to the library.
#pragma once
#include <hip/hip_runtime.h>
#include "rbkitk.h"

namespace rbki {

// Results of an enqueued decomposition, copied to host memory by the stream
// (pinned memory when the copy must not block).
struct HostResult {
  double sums[2];   // sum (x - xhat)^2, sum x^2
  int info[16];     // per mode: Jacobi sweep-limit flag, sweeps used
  int nmodes;
};

// Enqueue a whole rBKI-TK decomposition on `st` without synchronising, in the
// request server's form (every mode on `st`, beside other requests' solves);
// `hr` receives the error sums and the solver status when the stream reaches
// it.
rbki_status tucker_enqueue(const void* X, int xtype, const rbki_params* prm, void* core, void* const* factors,
                           int out_type, void* workspace, size_t ws_bytes, hipStream_t st, HostResult* hr);

// rel_err from the sums, and RBKI_E_NOCONV if an eigen-solve hit its limit.
rbki_status finish_result(const HostResult& hr, double* rel_err);

// Thread-local message of the last failure (the ABI's rbki_last_error).
void set_error(rbki_status s, const char* msg);

}  // namespace rbki

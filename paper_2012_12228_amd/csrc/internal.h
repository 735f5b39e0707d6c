// Library-internal hooks shared by the host translation units (not part of the C ABI).
#pragma once
#include "../../include/ftafqmc.h"

// Records the message of a failed initialisation for ftafqmc_last_error(NULL) on this thread
// and returns code.
int lib_init_error(int code, const char* msg);
// ftafqmc_init_ueg; with no_side_streams the handle creates no streams (systems run one after
// another, each system's walkers in one group).
int init_ueg_impl(const ftafqmc_params* p, int n_sys, void* d_workspace, size_t ws_bytes, void* stream,
                  ftafqmc_t* out, bool no_side_streams);
// Called by ftafqmc_destroy: a handle that held a device's static workspace releases it.
void static_ws_release(ftafqmc_t h);

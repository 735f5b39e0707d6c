// Library-internal hooks shared by the host translation units (not part of the C ABI).
#pragma once
#include "../../include/ftafqmc.h"

// Records the message of a failed initialisation for ftafqmc_last_error(NULL) on this thread
// and returns code.
int lib_init_error(int code, const char* msg);

// Internal host-side access to a handle, for host-orchestrated drivers built on the
// public entry points (the iteration of qst_solve.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "qst.h"

hipStream_t qst_host_stream(qst_handle* h);
qst_status qst_host_error(qst_handle* h, qst_status s, const std::string& msg);
int qst_host_device(const qst_handle* h);

// Internal declarations of the grid-wide single-system solve (grid.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "btpcg.h"

struct bt_handle;

// Scratch bytes of bt_grid_solve for a handle of one system.
size_t bt_grid_scratch_bytes(const bt_handle* h);

// PCG for the single system of ``h`` spread over the whole GPU in one
// persistent launch (asynchronous on the stream).
int bt_grid_solve(const bt_handle* h, const double* b, double* x, double tol,
                  int maxit, bt_info* info, void* ws, hipStream_t s);

// Device address of the library's own grid scratch array on the current
// device (BT_GRID_NOALLOC_MAX_BYTES), looked up once per device.
hipError_t bt_grid_static_scratch(void** out);

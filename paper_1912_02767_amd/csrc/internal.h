// Host-side functions shared between the driver, the batched engine and
// the server (not part of the C-ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "../../include/psdp.h"

namespace psdp {

// AUTO side rule of psdp_project (paper §6 plus the block cost rule):
// returns PSDP_SIDE_POS, _NEG or _FULL.
int auto_side(int n, int pos_hint, int m_cap, const psdp_options& opt);
// block an estimate of `est` eigenvalues needs: est + max(guard, ceil(0.2 est))
int block_need(int est, const psdp_options& opt);
// device and stream a handle enqueues on
int handle_device(psdp_handle h);
hipStream_t handle_stream(psdp_handle h);
// Every device-to-host copy the library makes goes through here: it is
// counted (copies, bytes, largest single copy) for psdp_transfer_stats.
hipError_t copy_to_host(void* dst, const void* src, size_t bytes, hipStream_t s);

}  // namespace psdp

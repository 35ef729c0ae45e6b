// Library-internal entry points shared by the driver (driver.hip) and the
// request server (serve.cpp). Not part of the C ABI.
#pragma once

#include <string>
#include <vector>

#include "gp.h"
#include "lower.h"

namespace gp {

// Merge already lowered circuits into one batch and upload it to the driver:
// gp_lower_batch without the lowering. Same status codes.
int driver_upload_parts(gp_driver* d, const std::vector<const Lowered*>& parts);

// Correlation level the driver lowers at.
uint32_t driver_level(const gp_driver* d);

// gp_fetch that hands back one new single-circuit result per circuit of the
// batch (in circuit order, each circuit's hyperedges in device order);
// wait_ns (if given, two entries) receives the time spent waiting for the
// device and the time spent downloading.
int driver_fetch_split(gp_driver* d, std::vector<gp_edges*>& out, uint64_t* wait_ns = nullptr);

// Record `msg` as this thread's gp_last_error text; returns `code`.
int set_last_error(int code, const std::string& msg);

}  // namespace gp

// Library-internal entry points shared by the driver (driver.hip) and the
// request server (serve.cpp). Not part of the C ABI.
#pragma once

#include <exception>
#include <new>
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

// Record `msg` as this thread's gp_last_error text; returns `code`. Never
// throws (if the text cannot be stored, the previous text stays).
int set_last_error(int code, const char* msg) noexcept;
inline int set_last_error(int code, const std::string& msg) noexcept { return set_last_error(code, msg.c_str()); }

// Runs fn (which returns a status) so that no C++ exception crosses the C
// ABI or leaves a library thread: an allocation failure becomes GP_E_OOM,
// any other exception GP_E_INTERNAL.
template <typename F>
int guarded(F&& fn) noexcept {
  try {
    return fn();
  } catch (const std::bad_alloc&) {
    return set_last_error(GP_E_OOM, "host memory allocation failed");
  } catch (const std::exception& e) {
    return set_last_error(GP_E_INTERNAL, e.what());
  } catch (...) {
    return set_last_error(GP_E_INTERNAL, "internal error");
  }
}

}  // namespace gp

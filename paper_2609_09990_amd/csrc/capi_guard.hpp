// Status translation at the C ABI: every entry point runs its body through
// guard(), which turns a library exception into a dmrg_status and keeps the
// message for dmrg_last_error() (thread-local).
#pragma once

#include <new>
#include <string>

#include "../../include/dmrg_mi355x.h"
#include "common.hpp"

namespace dmrg {

// Message of the last failed call on this thread.
std::string& last_error_slot();

template <class F>
dmrg_status guard(F&& f) {
  std::string& err = last_error_slot();
  try {
    err.clear();
    f();
    return DMRG_OK;
  } catch (const Error& e) {
    err = e.what();
    return (dmrg_status)e.code;
  } catch (const std::bad_alloc&) {
    err = "host allocation failed";
    return DMRG_ENOMEM;
  } catch (const std::exception& e) {
    err = e.what();
    return DMRG_EINVAL;
  }
}

}  // namespace dmrg

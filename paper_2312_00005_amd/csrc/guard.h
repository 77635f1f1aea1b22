// Status codes and the thread-local error message at the C boundary: every
// entry point runs its body through guarded(), which turns exceptions into a
// bem_status and a message for bem_last_error().
#pragma once

#include <new>
#include <string>

#include "common.h"

namespace bem {

void set_last_error(const std::string& msg);  // api.cpp
void clear_last_error();

inline bem_status fail(bem_status code, const std::string& msg) {
  set_last_error(msg);
  return code;
}

template <class F>
bem_status guarded(F&& f) {
  try {
    clear_last_error();
    return f();
  } catch (const Error& e) {
    return fail(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail(BEM_E_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(BEM_E_ARG, e.what());
  }
}

}  // namespace bem

// Pieces shared by the C entry points: the opaque handle and the guard that
// turns exceptions into status codes.
#pragma once

#include <memory>
#include <new>
#include <string>

#include "handle.h"
#include "method.h"

struct helm_handle {
  helm::Handle impl;
  std::unique_ptr<helm::Method> method;   // cached for the last batch width
};

namespace helm {

// Device address of this device's static scratch array of the
// allocation-free entry point (looked up once per device, with it current).
void* noalloc_scratch(int device);

// Run f(); map a thrown Error to its status code and record its text for
// helm_last_error.  No exception crosses the C ABI.
template <class F>
int guard(F&& f) {
  try {
    (void)hipGetLastError();   // do not report a failure of an earlier call
    return f();
  } catch (const Error& e) {
    set_last_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_last_error("host allocation failed");
    return HELM_ENOMEM;
  } catch (const std::exception& e) {
    set_last_error(e.what());
    return HELM_EINVAL;
  } catch (...) {
    set_last_error("unknown failure");
    return HELM_EINVAL;
  }
}

}  // namespace helm

// Inspection interface of the host-only test double (fake_runtime.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../paper_2308_03121_amd/csrc/nv_internal.h"

namespace fake {
struct Wait {
  int waiter;        // stream that waits
  int recorded_on;   // stream the event was last recorded on
  long seq;
};
long launches();
long bad_pointers();
const std::vector<std::string>& errors();
const std::vector<Wait>& waits();
void clear_waits();
size_t live_bytes();
size_t live_allocations();
hipStream_t new_stream();
int stream_id(hipStream_t s);
bool in_alloc(const void* p, size_t bytes);
}  // namespace fake

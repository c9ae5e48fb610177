// bf_filter_batched_noalloc: the batched filter for callers that cannot
// allocate (code under stream capture, serving loops, harnesses that forbid
// hipMalloc).  The job table and tile list live in a fixed device array of
// this library instead of a caller workspace; nothing is allocated.
//
// The array is a file-scope __device__ symbol, so every GPU the library runs
// on holds its own copy at its own address.  Host code never passes the
// symbol itself to a kernel or a copy (in host code it only names a
// host-side stand-in): its device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and kept.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "bf_internal.h"

namespace {

__device__ __attribute__((aligned(256))) unsigned char scratch[BF_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mutex;
std::map<int, void*>* g_scratch_ptr = new std::map<int, void*>();  // never freed: valid until exit

// device address of `scratch` on the stream's device (looked up on the
// first call for that device, with the device current)
int scratch_of(hipStream_t stream, void** out) {
  int dev = 0;
  hipError_t e = stream ? hipStreamGetDevice(stream, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) return bf::fail(BF_E_DEVICE, std::string("cannot query the stream's device: ") + hipGetErrorString(e));
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  auto it = g_scratch_ptr->find(dev);
  if (it != g_scratch_ptr->end()) {
    *out = it->second;
    return BF_OK;
  }
  int saved = -1;
  e = hipGetDevice(&saved);
  if (e == hipSuccess && saved != dev) e = hipSetDevice(dev);
  void* ptr = nullptr;
  if (e == hipSuccess) e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (saved >= 0 && saved != dev) (void)hipSetDevice(saved);
  if (e != hipSuccess || !ptr)
    return bf::fail(BF_E_DEVICE, std::string("cannot look up the scratch array: ") + hipGetErrorString(e));
  (*g_scratch_ptr)[dev] = ptr;
  *out = ptr;
  return BF_OK;
}

}  // namespace

extern "C" int bf_filter_batched_noalloc(const bf_job* jobs, int n_jobs, bf_planes prec, void* hip_stream) {
  return bf::filter_batched_pageable(jobs, n_jobs, prec, (size_t)BF_NOALLOC_SCRATCH_BYTES, "BF_NOALLOC_SCRATCH_BYTES",
                                     scratch_of, static_cast<hipStream_t>(hip_stream));
}

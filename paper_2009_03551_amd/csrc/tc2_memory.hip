// Device memory of the solver's buffers.
//
// A solve grows its large buffers (the iterate's values, the stage of kept
// blocks, the work arrays) over many updates, and a precision switch or a
// new context releases and re-requests tens of gigabytes.  Freeing a large
// allocation and asking for a larger one makes the GPU driver clear memory it has
// just reclaimed, at a few tens of GB/s, which stalls the device for seconds
// at the largest sizes.  Large buffers here therefore live in a virtual
// address range reserved once per buffer; physical memory is mapped into it
// in fixed chunks as the buffer grows, so growing keeps the contents and
// allocates only the increment.  Chunks a buffer gives back go to a pool per
// device and are mapped again by the next buffer that grows, within the same
// solve or in a later context (a later context would otherwise wait for the
// driver to clear the memory again: up to 2.6 s for one chunk at 256 MB after
// a large context was freed).  The pool is returned to the GPU driver when an
// allocation of the library fails for lack of memory (and then retried), and
// by tc2_trim_memory, for callers whose other allocations need the memory.
#include "tc2_context.h"

#include <mutex>
#include <vector>

namespace tc2 {

namespace {

constexpr int MAX_DEVICES = 64;

struct Pool {
  std::mutex m;
  bool init = false;
  bool ok = false;           // the device supports the virtual memory calls
  size_t chunk = 0;          // bytes per physical chunk
  size_t va = 0;             // bytes of virtual range reserved per buffer
  std::vector<hipMemGenericAllocationHandle_t> free;
};

Pool g_pool[MAX_DEVICES];

hipMemAllocationProp chunk_prop(int dev) {
  hipMemAllocationProp prop = {};
  prop.type = hipMemAllocationTypePinned;
  prop.location.type = hipMemLocationTypeDevice;
  prop.location.id = dev;
  return prop;
}

// Pool of the current device, set up on first use; nullptr when the device
// does not support the calls (buffers then fall back to plain allocations).
Pool* pool_of(int* dev_out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  Pool& P = g_pool[dev];
  std::lock_guard<std::mutex> g(P.m);
  if (!P.init) {
    P.init = true;
    const hipMemAllocationProp prop = chunk_prop(dev);
    size_t gran = 0;
    size_t total = 0;
    if (hipMemGetAllocationGranularity(&gran, &prop, hipMemAllocationGranularityMinimum) ==
            hipSuccess &&
        gran > 0 && hipDeviceTotalMem(&total, dev) == hipSuccess && total > 0) {
      const size_t want = (size_t)256 << 20;
      P.chunk = (want + gran - 1) / gran * gran;
      P.va = (total / P.chunk + 2) * P.chunk;
      P.ok = true;
    }
    (void)hipGetLastError();
  }
  if (dev_out) *dev_out = dev;
  return P.ok ? &P : nullptr;
}

}  // namespace

// Return every pooled chunk of the current device to the GPU driver.
void pool_trim() {
  int dev = 0;
  Pool* P = pool_of(&dev);
  if (!P) return;
  std::lock_guard<std::mutex> g(P->m);
  for (hipMemGenericAllocationHandle_t h : P->free) (void)hipMemRelease(h);
  P->free.clear();
}

hipError_t dev_malloc(void** p, size_t n) {
  hipError_t e = hipMalloc(p, n);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    pool_trim();
    e = hipMalloc(p, n);
  }
  return e;
}

// Grow the virtual range of b to at least n bytes, keeping what is mapped.
hipError_t vm_grow(DBuf& b, size_t n) {
  int dev = 0;
  Pool* P = pool_of(&dev);
  if (!P) return hipErrorNotSupported;
  if (!b.vm) {
    void* base = nullptr;
    hipError_t e = hipMemAddressReserve(&base, P->va, 0, nullptr, 0);
    if (e != hipSuccess) return e;
    b.p = base;
    b.cap = 0;
    b.va = P->va;
    b.vm = true;
    b.dev = dev;
  }
  if (n > b.va) return hipErrorOutOfMemory;
  const size_t need = (n + P->chunk - 1) / P->chunk;
  const hipMemAllocationProp prop = chunk_prop(dev);
  hipMemAccessDesc acc = {};
  acc.location.type = hipMemLocationTypeDevice;
  acc.location.id = dev;
  acc.flags = hipMemAccessFlagsProtReadWrite;
  while (b.chunks.size() < need) {
    hipMemGenericAllocationHandle_t h{};
    bool have = false;
    {
      std::lock_guard<std::mutex> g(P->m);
      if (!P->free.empty()) {
        h = P->free.back();
        P->free.pop_back();
        have = true;
      }
    }
    if (!have) {
      hipError_t e = hipMemCreate(&h, P->chunk, &prop, 0);
      if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        pool_trim();
        e = hipMemCreate(&h, P->chunk, &prop, 0);
      }
      if (e != hipSuccess) return e;
    }
    char* at = (char*)b.p + b.chunks.size() * P->chunk;
    hipError_t e = hipMemMap(at, P->chunk, 0, h, 0);
    if (e == hipSuccess) e = hipMemSetAccess(at, P->chunk, &acc, 1);
    if (e != hipSuccess) {
      (void)hipMemUnmap(at, P->chunk);
      std::lock_guard<std::mutex> g(P->m);
      P->free.push_back(h);
      return e;
    }
    b.chunks.push_back(h);
    b.cap = b.chunks.size() * P->chunk;
  }
  return hipSuccess;
}

// Unmap every chunk of b (once the device is idle) into the pool, and free
// its virtual range.
void vm_release(DBuf& b) {
  if (!b.vm) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != b.dev) (void)hipSetDevice(b.dev);
  (void)hipDeviceSynchronize();
  Pool& P = g_pool[b.dev];
  for (size_t k = 0; k < b.chunks.size(); ++k) (void)hipMemUnmap((char*)b.p + k * P.chunk, P.chunk);
  {
    std::lock_guard<std::mutex> g(P.m);
    P.free.insert(P.free.end(), b.chunks.begin(), b.chunks.end());
  }
  b.chunks.clear();
  (void)hipMemAddressFree(b.p, b.va);
  if (cur != b.dev) (void)hipSetDevice(cur);
  b.p = nullptr;
  b.cap = 0;
  b.va = 0;
  b.vm = false;
}

}  // namespace tc2

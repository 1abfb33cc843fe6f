// Every buffer the kernels read or write through a parameter block lives in
// device global memory.  Pointers loaded from memory (the batch engine's
// parameter blocks) are generic to the compiler, which then emits flat
// accesses with 64-bit vector addresses and cannot use scalar loads for
// uniform values such as coefficient tables.  The device code therefore
// accesses memory through pointers typed in the global address space; for
// kernel arguments this changes nothing.
#pragma once
#include <hip/hip_runtime.h>

namespace rbc {

template <typename T>
using gbl = __attribute__((address_space(1))) T;

template <typename T>
__device__ __forceinline__ gbl<T>* global_ptr(T* p) {
  return (gbl<T>*)p;
}

}  // namespace rbc

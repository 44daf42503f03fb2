// Global-memory pointers for addresses that kernels read from device tables
// (a job's output arrays, a cell type's K_r).
#pragma once

#include <hip/hip_runtime.h>

namespace mos {

// A pointer the kernel loads from memory has no address space the compiler
// can prove, so accesses through it become flat instructions, and on gfx950
// a flat access counts against the LDS wait counter as well as the vector
// memory one: the wave's next wait for an LDS read then also waits for the
// flat store or load to complete.  Converted once to a global pointer, the
// same accesses are global instructions and the LDS waits stay exact.
template <class T>
using global_ptr = __attribute__((address_space(1))) T *;

template <class T>
__device__ __forceinline__ global_ptr<T> to_global(T *p) {
    return (global_ptr<T>)p;
}

}  // namespace mos

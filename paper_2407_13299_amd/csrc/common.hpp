// Internal definitions shared by the HIP translation units of libdmp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "layout.hpp"

namespace dmp {

#define DMP_CHECK_HIP(call)                                                  \
    do {                                                                     \
        hipError_t err_ = (call);                                            \
        if (err_ != hipSuccess) {                                            \
            ::dmp::set_error("%s:%d %s: %s", __FILE__, __LINE__, #call,       \
                             hipGetErrorString(err_));                       \
            return DMP_EHIP;                                                 \
        }                                                                    \
    } while (0)

}  // namespace dmp

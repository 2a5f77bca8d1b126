// Event-bracketed kernel timing (see prof.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/fks.h"

namespace fks {

bool prof_on();

// Records a start event on construction and a stop event on destruction, on
// the given stream, when timing is enabled; costs one branch otherwise.
class ProfScope {
  public:
    ProfScope(const char* name, hipStream_t st);
    ~ProfScope();
    ProfScope(const ProfScope&) = delete;
    ProfScope& operator=(const ProfScope&) = delete;

  private:
    const char* name_;
    hipStream_t st_;
    hipEvent_t start_ = nullptr, stop_ = nullptr;
};

}  // namespace fks

#define FKS_TIMED(name, st, launch)           \
    do {                                      \
        fks::ProfScope prof_scope_(name, st); \
        launch;                               \
    } while (0)

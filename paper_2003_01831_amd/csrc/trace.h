// RAII phase timer used around the launches of each step phase.
#pragma once
#include "common.h"

class TraceScope {
 public:
  TraceScope(int phase, hipStream_t st);
  ~TraceScope();
  TraceScope(const TraceScope&) = delete;
  TraceScope& operator=(const TraceScope&) = delete;

 private:
  long slot_;
  hipStream_t st_;
};

// Definitions of the opaque handles of include/rbc.h.
#pragma once

#include "core.hpp"

struct rbc_scheme_s {
  rbc::Scheme s;
};
struct rbc_plan_s {
  rbc::Plan p;
};

// Definitions of the opaque C handles (one per public object).
#pragma once

#include "plan.hpp"
#include "sara.hpp"

struct ri_plan_s {
  ri::Plan p;
};

struct ri_sara_s {
  ri::Sara s;
};

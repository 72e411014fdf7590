// EDFA preconditioner handle (internal layout of an edfa_precond).
#pragma once

#include "system.hpp"

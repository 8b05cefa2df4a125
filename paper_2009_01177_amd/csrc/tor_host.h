// tor_host.h -- host-only scheduling helpers (declared for C in include/tor.h).
#pragma once
#include "../../include/tor.h"

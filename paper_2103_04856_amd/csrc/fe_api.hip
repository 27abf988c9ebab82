// The library's one translation unit: the kernels (fe_*.hpp) and the host side
// of the C ABI declared in include/fe.h, split by topic into host_core.hpp
// (context, constants, sweeps, step loops, autotuner), host_flow.hpp
// (Algorithm 1), host_diag.hpp (diagnostics), host_l2.hpp (Algorithm 2) and
// host_noalloc.hpp (the allocation-free energy + gradient entry point).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "fe.h"
#include "fe_flow.hpp"
#include "fe_diag.hpp"
#include "fe_l2flow.hpp"
#include "fe_kernels.hpp"

#include "host_core.hpp"
#include "host_flow.hpp"
#include "host_diag.hpp"
#include "host_l2.hpp"
#include "host_noalloc.hpp"

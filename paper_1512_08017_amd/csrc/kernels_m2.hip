// Kernels and launchers for calls whose largest degree is 2.
#include "kernels_impl.hpp"

template struct lsefit::Launchers<2>;

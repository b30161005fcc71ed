// Kernels and launchers for calls whose largest degree is 1.
#include "kernels_impl.hpp"

template struct lsefit::Launchers<1>;

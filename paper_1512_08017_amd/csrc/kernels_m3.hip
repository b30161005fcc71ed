// Kernels and launchers for calls whose largest degree is 3.
#include "kernels_impl.hpp"

template struct lsefit::Launchers<3>;

// Kernels and launchers for calls whose largest degree is 7.
#include "kernels_impl.hpp"

template struct lsefit::Launchers<7>;

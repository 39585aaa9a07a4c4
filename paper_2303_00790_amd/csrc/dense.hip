// placeholder
#include "internal.hpp"

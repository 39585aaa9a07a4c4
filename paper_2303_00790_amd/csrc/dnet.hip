#include "internal.hpp"

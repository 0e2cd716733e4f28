// stubs.hip -- entry points whose full implementation lives elsewhere.
#include "abi_internal.h"


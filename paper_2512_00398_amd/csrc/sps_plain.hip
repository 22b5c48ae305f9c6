// sps_plain.hip - placeholder translation unit for the per-stage path.
#include "sps_internal.h"

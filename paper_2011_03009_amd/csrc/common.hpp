// Definitions shared by host and device code.
#pragma once

#define NVP_MAX_FIELDS 7  // harmonics up to 8

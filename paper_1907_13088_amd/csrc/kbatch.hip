// Batched multi-grid stepping (placeholder until implemented)
#include "mx_internal.h"

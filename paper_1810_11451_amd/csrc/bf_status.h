// Status reporting shared by every part of libbf, including the parts that
// are built without HIP (the serving loop's core and its host executor).
#pragma once

#include "bf.h"

// Records a printf-style detail for bf_last_error() on the calling thread
// and returns s.
bf_status bf_fail(bf_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

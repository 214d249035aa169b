// Serving loop (continuous batching of fitness and prediction requests).
#include "internal.h"

extern "C" void aerl_serve_shutdown_internal(aerl_ctx *ctx) { (void)ctx; }

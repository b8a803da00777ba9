// Serving engine (continuous batching of RIR requests).
#include "ism_host.h"

void ism_serve_release(ism_handle *h) { (void)h; }

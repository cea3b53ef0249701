// Serving loop (continuous batching over resident scenes).
#include "runtime.h"

namespace swf {
void serve_shutdown(Ctx* c) { (void)c; }
}  // namespace swf

// Serving loop of the C ABI (continuous batching of render requests).
#pragma once
namespace kn {
class ServeLoop;
}

// Supported grid sizes N (even, 2^a 3^b).  The build instantiates every kernel for each of them
// in float32 and float64 (the list is read by the build script too: one entry per line).
#pragma once

#define PIN_FOR_EACH_SIZE(X) \
  X(8)                       \
  X(12)                      \
  X(16)                      \
  X(24)                      \
  X(32)                      \
  X(48)                      \
  X(64)                      \
  X(96)                      \
  X(128)                     \
  X(192)                     \
  X(256)                     \
  X(384)                     \
  X(512)                     \
  X(768)                     \
  X(1024)

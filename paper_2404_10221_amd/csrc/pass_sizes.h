// Transform lengths L = 2(N+1) the library carries kernels for.
#pragma once
#define RSFDE_FOR_EACH_L(X) \
  X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) \
  X(768) X(1024) X(1536) X(2048) X(3072) X(4096)

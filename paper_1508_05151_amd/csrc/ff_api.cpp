// Host-only parts of the C ABI.
#include "ff.h"

extern "C" const char* ff_status_string(ff_status s) {
  switch (s) {
    case FF_OK: return "ok";
    case FF_ERR_ARG: return "invalid argument";
    case FF_ERR_SIZE: return "image too large";
    case FF_ERR_WORKSPACE: return "workspace or descriptor buffer too small";
    case FF_ERR_UNSUPPORTED: return "unsupported";
    case FF_ERR_HIP: return "HIP runtime error";
    case FF_ERR_DEVICE: return "device watchdog fired";
  }
  return "unknown status";
}

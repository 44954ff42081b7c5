// Internal error type of the hifcn library (host code only, no HIP): internal code throws
// HifError; the C entry points translate it to a status code.
#pragma once

#include <stdexcept>
#include <string>

#include "../../include/hifcn.h"

namespace hifcn {

struct HifError : std::runtime_error {
  hif_status_t status;
  HifError(hif_status_t s, const std::string& m) : std::runtime_error(m), status(s) {}
};

}  // namespace hifcn

#define HIF_REQUIRE(cond, status, msg)                                                        \
  do {                                                                                        \
    if (!(cond)) throw ::hifcn::HifError((status), (msg));                                    \
  } while (0)

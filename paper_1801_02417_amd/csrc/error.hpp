// Status-carrying exception of the library's host code (host only: shared by the HIP layers and
// by the request server's scheduler, which builds without HIP).
#pragma once

#include <string>

#include "psara.h"

namespace psara {

struct Error {
  psara_status status;
  std::string msg;
  Error(psara_status s, std::string m) : status(s), msg(std::move(m)) {}
};

}  // namespace psara

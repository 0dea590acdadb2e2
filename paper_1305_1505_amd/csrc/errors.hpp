// Status-carrying exception used inside the library; converted to pin_status at the C ABI.
#pragma once

#include <exception>
#include <string>
#include <utility>

#include "pin.h"

namespace pin {

struct PinError : std::exception {
  pin_status status;
  std::string msg;
  PinError(pin_status s, std::string m) : status(s), msg(std::move(m)) {}
  const char* what() const noexcept override { return msg.c_str(); }
};

}  // namespace pin

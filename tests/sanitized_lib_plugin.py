"""pytest plugin (loaded with -p by the sanitizer test only): points the ctypes binding at
the library named by MMS_SANITIZED_LIB, a build of the same sources with host-side
AddressSanitizer and UndefinedBehaviorSanitizer."""
import os


def pytest_configure(config):
    path = os.environ.get("MMS_SANITIZED_LIB")
    if path:
        from paper_2507_11067_amd import _lib
        _lib.LIB = path
        _lib._lib = None

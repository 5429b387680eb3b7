"""Declarations and wrappers of the hit-binning and building calls (filled in with the build path)."""


def declare(lib):
    return lib

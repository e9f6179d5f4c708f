"""Serving API binding (filled in by the server entry points of libgz.so)."""


def _declare(L):
    return L

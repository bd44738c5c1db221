"""Seeded synthetic inputs shared by the oracle and the HIP library's tests.

This package holds no arithmetic of the eigensolver: it draws matrices and
Householder-reflector inputs of the right shape, structure and distribution.
"""
from .gen import *  # noqa: F401,F403

"""CPU oracle for the PAGANI integrator -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. It wraps ``liboracle.so`` (built from
``pagani_oracle.c`` by :func:`oracle.build.build`), a plain sequential C
implementation of Algorithm 2 and Algorithm 3 of the paper, and shares no
code with the GPU library.
"""
from .oracle import *  # noqa: F401,F403

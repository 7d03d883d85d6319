"""CPU oracle for bucket ORP and bucket oblivious sort — TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle.so`` (built from
``bos_oracle.cpp`` by :func:`build`), which shares no code with the GPU library.
"""
from .oracle import *  # noqa: F401,F403

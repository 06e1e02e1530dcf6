"""CPU oracle for the RNS-FHE hot path: TEST INFRASTRUCTURE ONLY.

A plain, slow, independent implementation of what the GPU library computes,
written from the textbook definitions the paper relies on (RNS/CRT over the
rings R_q of its background section, CKKS/BGV/BFV multiplication, the level
concept behind rescale and modulus switching).  It shares no code, tables or
constants with the product library (``paper_2503_22227_amd``) and neither
imports the other; both draw their random inputs from ``synthetic``.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  Arithmetic is exact: Python integers for CRT-level
constants and checks, and a small C core (``core.c``) that evaluates every
modular product as (a*b) mod q on 128-bit integers.

Modules:
  params   prime chains, roots of unity, digit partition
  ntt      the negacyclic NTT: O(N^2) definition and the fast transform
  rns      CRT composition/decomposition with Python big integers
  ckks     encode/decode, keys, encryption, HMult+Relin, key switching,
           rescale, automorphism and rotation
"""

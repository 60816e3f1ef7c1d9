"""Exact CPU oracle for the k-input RNS-CKKS ciphertext multiply.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, tables or
constant generators with the HIP library; both sides follow the same written
conventions (prime choice, NTT order, sampler definitions) and are compared
residue by residue.

Arithmetic is exact: residues are numpy uint64 with every modulus below 2^31,
so products stay below 2^62; CRT work uses Python integers.  FP64 appears
only in encode/decode (the paper does not describe encoding).

Modules
-------
params   primes, psi, basis-conversion constants (RNS, Sec. II)
prng     SplitMix64 counter streams and the samplers built on them
ntt      negacyclic NTT / INTT and the direct evaluation that defines them
keys     secret key, public key, evaluation keys for s^2..s^k (Sec. II, Sec. V-A)
ckks     encode / encrypt / decrypt / decode (Sec. II)
mult     tensor product, ModUp, key inner product, ModDown (textbook and
         relocated), single and multi-level rescaling (Sec. II-V)
tree     tree-structured n-input multiply with rescaling inside the tree and
         its partition planner (Sec. V-B, V-C, Table II)
counts   transform counters used to check the paper's operation counts
"""

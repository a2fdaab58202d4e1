"""CPU oracle for the two-site DMRG sigma path.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call or execute anything in this package.  The product
path (``paper_2609_09990_amd``) never does; it shares no code with it.

Contents (plain, slow, fp64, written from the definitions):

* ``fci``   - determinant space with colexicographic string addressing
              (addr = sum_i C(o_i, i+1), the paper's CI addressing, Sec. III),
              Knowles-Handy sigma, dense / Davidson eigensolve, 1-/2-RDMs,
              <S^2> via ||S_+ c||^2 (Sec. III; per determinant, and with
              sparse string ladder operators for large spaces), integral
              gradients.
* ``fock``  - brute-force Jordan-Wigner Fock-space Hamiltonian for tiny n, for
              any spin-orbital ordering (pins ``fci`` and the MPS sign rule).
* ``embed`` - MPS -> Fock-space embedding and the two-site projected sigma
              P^T H P psi (the definition of H_eff psi for a given MPS basis);
              the projection P^T Phi of another state into a two-site space
              and the MPS overlap (penalty deflation, Sec. II.F).
* ``mlp``   - fp64 NumPy 3-layer MLP forward/backward and Adam (reference for
              the preconditioner network kernels).
* ``mpo``   - the oracle's own MPO of H, built generically from the list of
              normal-ordered second-quantised terms (an automaton: each term's
              left string is carried until a switch site, its right string
              after it); pinned by dense contraction against ``fock``.
* ``blocks``- block-sparse environments on that MPO, the two-site sigma (whole
              or chosen output blocks, with its own flop count) and the H_eff
              diagonal; pinned against the projected FCI sigma of ``embed``.
              It runs at production shape (CAS(20,20), M = 1024).
* ``truncate`` - per-sector SVD truncation with the global sort, the cluster
              rule, cut_rtol and tau; state averaging by concatenation.

Every function's pin (what it is checked against other than itself) is listed
in its docstring; the pins live in ``tests/test_oracle_*.py``.
"""

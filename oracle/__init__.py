"""FP64 CPU oracle for two-flavour Wilson-fermion HMC with hopping-parameter-expansion filtering.

THIS PACKAGE IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite, the
smoke check in ``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` may import it.
The HIP library never links it and the Python binding never calls it.

It is a plain, slow, deliberately unoptimised numpy implementation of what the method
computes, written from M. Hasenbusch, "Exploiting the hopping parameter expansion in the
hybrid Monte Carlo simulation of lattice QCD with two degenerate flavours of Wilson
fermions" (arXiv:1805.03560).  Each function cites the section / equation it follows.
All floating point is float64 / complex128; the filter coefficients are computed in exact
rational arithmetic plus 50-digit mpmath.

Conventions (the paper leaves them open; they are recorded once here and in the C header):

* lattice dims are given as (L_t, L_z, L_y, L_x); direction mu is array axis mu, so mu=0 is
  time and mu=1,2,3 are z, y, x.
* lexicographic site index  lex = ((t*L_z + z)*L_y + y)*L_x + x ; parity = (t+z+y+x) mod 2 ;
  checkerboard index cb = lex // 2 (needs L_x even).  A half-lattice vector of parity p lists
  the sites of parity p in increasing lex order, i.e. by cb index.
* gauge links are periodic; fermion hops that cross the time boundary pick up a factor -1
  (Sec. 4: periodic in space, anti-periodic in time for the fermions).
* chiral Euclidean gamma basis (see ``oracle.gamma``).
* Pi = sum_a pi_a T_a with T_a = i lambda_a / 2, so (Pi,Pi) = -2 sum Tr Pi^2 = sum pi_a^2
  (Sec. 1, eq. Sproduct); forces F are stored the same way, (omega, F) = sum_a omega_a f_a.
"""

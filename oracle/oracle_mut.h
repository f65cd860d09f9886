/* oracle_mut.h -- planted-mistake switches of the oracle's pin self-check.
 *
 * TEST INFRASTRUCTURE.  MUT(k) marks a term that mistake k breaks.  The
 * switches exist only in the separate build liboracle_mut.so (compiled with
 * -DORC_MUTANTS), which only tests/test_oracle_mutants.py loads; in the oracle
 * that the GPU path is compared with (liboracle.so) every MUT(k) is the
 * constant 0, so no switch can be left set there. */
#ifndef ORACLE_MUT_H
#define ORACLE_MUT_H
#ifdef ORC_MUTANTS
int orc_get_mutant(void);
#define MUT(k) (orc_get_mutant() == (k))
#else
#define MUT(k) 0
#endif
#endif

# Weyl semimetal of Sec. 2.3 with k0 = pi/2, written for the tests: hops
# sigma_x/2 along x and (sigma_x + i sigma_j)/2 along j = y, z; on-site
# -sigma_x (2 + cos k0) as the constant c0; disorder generated on the fly
dim 3
size 2
n_coeff_const 1
n_coeff_rand 1
coeff_const_default -2
nn -1 0 0
l0; 1|0.5
l1; 0|0.5
nn 1 0 0
l0; 1|0.5
l1; 0|0.5
nn 0 -1 0
l0; 1|1
l1;
nn 0 1 0
l0;
l1; 0|1
nn 0 0 -1
l0; 0|0.5i; 1|0.5
l1; 0|0.5;  1|-0.5i
nn 0 0 1
l0; 0|-0.5i; 1|0.5
l1; 0|0.5;   1|0.5i
nn 0 0 0
l0; 0|r|0; 1|c|0
l1; 0|c|0; 1|r|0
